// Bit-matrix utility kernels: packing (ingest), decoding, element-wise
// Boolean operators, transpose, padding checks and bits -> CSR.
//
// Layout everywhere: row-major, LSB-first uint64 words; column j of row i is
// bit (j & 63) of word i*ld + (j >> 6).  This is the paper's row encoding of a
// relation as facts v(i, b_i) whose code b_i has bit j set iff r(c_i, c_j)
// (Section 3.2), with the code split into 64-bit words.
#include "bmlp_internal.h"

#include <algorithm>
#include <type_traits>

namespace bmlp {

namespace {

constexpr int kBlock = 256;

inline int grid_for(i64 work, int per_block = kBlock, int cap = 65536) {
  i64 g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__device__ inline u64 last_word_mask(i64 n) {
  int r = (int)(n & 63);
  return r == 0 ? ~0ull : ((1ull << r) - 1ull);
}

__global__ void k_fill_zero(u64* __restrict__ p, i64 nwords) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < nwords; i += (i64)gridDim.x * blockDim.x) p[i] = 0;
}

// Seeded random bits for the autotuner's synthetic operands: every bit of word (row, w) is 1 with
// probability 2^-s (the AND of s words of a counter-based hash, splitmix64's finaliser), s = s_in inside
// the block rows < brows, words < bwords and s_out elsewhere; padding bits stay 0.
__device__ __forceinline__ u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_fill_random(u64* __restrict__ a, i64 rows, i64 n, i64 ld, u64 seed, int s_in, int s_out, i64 brows,
                              i64 bwords) {
  const i64 nw = (n + 63) >> 6;
  const i64 total = rows * ld;
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x) {
    const i64 row = i / ld, w = i - row * ld;
    u64 v = 0;
    if (w < nw) {
      const int sh = (row < brows && w < bwords) ? s_in : s_out;
      v = ~0ull;
      for (int k = 0; k < sh; ++k) v &= mix64(seed + 0x9E3779B97F4A7C15ull * (u64)(i * 16 + k + 1));
      if (w == nw - 1) v &= last_word_mask(n);
    }
    a[i] = v;
  }
}

// one wave per output word: lane l looks at byte (row, 64w + l); the wave
// ballot is the packed word.
__global__ void k_pack_u8(const uint8_t* __restrict__ d, i64 rows, i64 n, i64 ldd, u64* __restrict__ bits, i64 ld) {
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  const i64 total = rows * ld;
  for (i64 wi = wave; wi < total; wi += nwaves) {
    const i64 row = wi / ld, w = wi - row * ld;
    const i64 col = w * 64 + lane;
    int v = 0;
    if (col < n) v = d[row * ldd + col] != 0;
    u64 word = __ballot(v);
    if (lane == 0) bits[wi] = word;
  }
}

__global__ void k_unpack_u8(const u64* __restrict__ bits, i64 rows, i64 n, i64 ld, uint8_t* __restrict__ d, i64 ldd) {
  const i64 total = rows * n;
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    const i64 row = t / n, col = t - row * n;
    d[row * ldd + col] = (uint8_t)((bits[row * ld + (col >> 6)] >> (col & 63)) & 1ull);
  }
}

__global__ void k_pack_coo(const int32_t* __restrict__ r, const int32_t* __restrict__ c, i64 m, i64 rows, i64 n,
                           u64* __restrict__ bits, i64 ld, u32* __restrict__ bad) {
  for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
    const int32_t i = r[e], j = c[e];
    if (i < 0 || i >= rows || j < 0 || j >= n) {
      atomicOr(bad, 1u);
      continue;
    }
    atomicOr((unsigned long long*)&bits[(i64)i * ld + (j >> 6)], 1ull << (j & 63));
  }
}

__global__ void k_ewise(int op, const u64* __restrict__ a, i64 lda, const u64* __restrict__ b, i64 ldb,
                        u64* __restrict__ c, i64 ldc, i64 rows, i64 n, const u32* __restrict__ pred, u32 pred_val) {
  if (pred && *pred != pred_val) return;
  const i64 nw = (n + 63) >> 6;
  const i64 total = rows * ldc;
  const u64 lm = last_word_mask(n);
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    const i64 row = t / ldc, w = t - row * ldc;
    u64 v = 0;
    if (w < nw) {
      const u64 x = a[row * lda + w];
      switch (op) {
        case 0: v = x | b[row * ldb + w]; break;
        case 1: v = x & b[row * ldb + w]; break;
        case 2: v = x & ~b[row * ldb + w]; break;
        case 3: v = ~x; break;
        default: v = x; break;
      }
      if (w == nw - 1) v &= lm;
    }
    c[t] = v;
  }
}

__global__ void k_zero_pad(u64* __restrict__ a, i64 rows, i64 nw, i64 ld) {
  const i64 pw = ld - nw;
  const i64 total = rows * pw;
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    const i64 row = t / pw, w = nw + (t - row * pw);
    a[row * ld + w] = 0ull;
  }
}

__global__ void k_set_diag(u64* __restrict__ a, i64 ld, i64 cnt) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < cnt; i += (i64)gridDim.x * blockDim.x)
    a[i * ld + (i >> 6)] |= 1ull << (i & 63);
}

// row i gets the single bit idx[i] (rows zeroed beforehand)
// row i of a (zeroed by the caller) gets the single bit idx[i]; an index outside [0, n) is skipped and
// raises *bad
__global__ void k_set_onehot(u64* __restrict__ a, i64 ld, const int32_t* __restrict__ idx, i64 k, i64 n,
                             u32* __restrict__ bad) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < k; i += (i64)gridDim.x * blockDim.x) {
    const i64 j = idx[i];
    if (j < 0 || j >= n) {
      if (bad) atomicOr(bad, 1u);
      continue;
    }
    a[i * ld + (j >> 6)] = 1ull << (j & 63);
  }
}

// row index of every entry of a CSR layout: out[rp[r] .. rp[r+1]) = r, one wave per row
__global__ void k_rows_from_rp(const i64* __restrict__ rp, i64 rows, int32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  for (i64 r = wave; r < rows; r += nwaves)
    for (i64 e = rp[r] + lane; e < rp[r + 1]; e += 64) out[e] = (int32_t)r;
}

// list of the rows of a with a set bit (order unspecified), *count = their number.  A wave takes eight rows
// with all their loads in flight and claims their slots in the list with one atomic (one same-address
// atomic per row, each waited for, took 55 us for 16,384 rows).
__global__ void k_nonempty_rows(const u64* __restrict__ a, i64 rows, i64 nw, i64 ld, int32_t* __restrict__ list,
                                u32* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  for (i64 r0 = wave * 8; r0 < rows; r0 += nwaves * 8) {
    u64 any[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) any[q] = 0ull;
    for (i64 w = lane; w < nw; w += 64) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (r0 + q < rows) any[q] |= a[(r0 + q) * ld + w];
    }
    u32 mask = 0;  // wave-uniform: bit q = row r0 + q has a set bit
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (__ballot(any[q] != 0ull)) mask |= 1u << q;
    u32 base = 0;
    if (lane == 0 && mask) base = atomicAdd(count, (u32)__popc(mask));
    base = __shfl(base, 0, 64);
    if (lane < 8 && ((mask >> lane) & 1u)) list[base + (u32)__popc(mask & ((1u << lane) - 1u))] = (int32_t)(r0 + lane);
  }
}

// dst row i = src row list[i] (nw words), one wave per row
__global__ void k_copy_rows(const u64* __restrict__ src, i64 lds, const int32_t* __restrict__ list, i64 k, i64 nw,
                            u64* __restrict__ dst, i64 ldd) {
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  for (i64 i = wave; i < k; i += nwaves) {
    const i64 r = list[i];
    for (i64 w = lane; w < ldd; w += 64) dst[i * ldd + w] = w < nw ? src[r * lds + w] : 0ull;
  }
}

// One-hot queries answered from a closure: out row i = C row idx[i] (| bit idx[i] when reflexive), padding
// words up to ldo zeroed; an index outside [0, n) gives a zero row and raises *bad.  A workgroup copies
// 1,024 words of one row (segment seg of row i), four words per thread with all four loads in flight, so
// that a query of few rows waits for one memory round trip rather than one per 512 bytes.
constexpr int kRowSegWords = 4 * kBlock;
__global__ void __launch_bounds__(kBlock)
k_rows_by_index(const u64* __restrict__ C, i64 ldc, const int32_t* __restrict__ idx, i64 k, i64 n, int reflexive,
                u64* __restrict__ out, i64 ldo, u32* __restrict__ bad) {
  const i64 nw = (n + 63) >> 6;
  const i64 segs = (ldo + kRowSegWords - 1) / kRowSegWords;
  for (i64 b = blockIdx.x; b < k * segs; b += gridDim.x) {
    const i64 i = b / segs, w0 = (b - i * segs) * kRowSegWords;
    const i64 j = idx[i];
    const bool ok = j >= 0 && j < n;
    if (!ok && w0 == 0 && threadIdx.x == 0 && bad) atomicOr(bad, 1u);
    u64 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const i64 w = w0 + q * kBlock + threadIdx.x;
      v[q] = (ok && w < nw) ? C[j * ldc + w] : 0ull;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const i64 w = w0 + q * kBlock + threadIdx.x;
      if (ok && reflexive && w == (j >> 6)) v[q] |= 1ull << (j & 63);
      if (w < ldo) out[i * ldo + w] = v[q];
    }
  }
}

// raises *bad when an index lies outside [0, n)
__global__ void k_check_index(const int32_t* __restrict__ idx, i64 k, i64 n, u32* __restrict__ bad) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < k; i += (i64)gridDim.x * blockDim.x) {
    const i64 j = idx[i];
    if (j < 0 || j >= n) atomicOr(bad, 1u);
  }
}

// Column gather: A[x][i] = T[x][cols[i]] (| (cols[i] == x) when diag), one workgroup per row x of T
// with the row staged in LDS; each wave turns 64 consecutive i into one word of A by a ballot.
__global__ void __launch_bounds__(256)
k_gather_cols(const u64* __restrict__ T, i64 ldt, i64 rows, i64 n, const int32_t* __restrict__ cols, i64 b,
              int diag, u64* __restrict__ A, i64 lda) {
  extern __shared__ u64 rowbuf[];
  const i64 nw = (n + 63) >> 6, bw = (b + 63) >> 6;
  const int t = threadIdx.x, lane = t & 63;
  for (i64 x = blockIdx.x; x < rows; x += gridDim.x) {
    for (i64 w = t; w < nw; w += 256) rowbuf[w] = T[x * ldt + w];
    __syncthreads();
    for (i64 i0 = (i64)(t >> 6) * 64; i0 < b; i0 += 256) {
      const i64 i = i0 + lane;
      int bit = 0;
      if (i < b) {
        const i64 c = cols[i];
        bit = (int)((rowbuf[c >> 6] >> (c & 63)) & 1ull) | (diag && c == x ? 1 : 0);
      }
      const u64 word = __ballot(bit);
      if (lane == 0) A[x * lda + (i0 >> 6)] = word;
    }
    for (i64 w = bw + t; w < lda; w += 256) A[x * lda + w] = 0ull;
    __syncthreads();  // the row buffer is refilled for the next row
  }
}

// I | M+ for a relation of b <= 64 nodes (one word per row), by Warshall's algorithm in one wave: lane
// i holds row i; at step k every row with bit k set takes in row k (read by a shuffle, so it already
// holds the paths through nodes < k).
__global__ void k_closure64(const u64* __restrict__ M, i64 ldm, i64 b, u64* __restrict__ out, i64 ldo) {
  const int lane = threadIdx.x & 63;
  const u64 mask = b >= 64 ? ~0ull : ((1ull << b) - 1ull);
  u64 row = lane < b ? (M[lane * ldm] & mask) : 0ull;
  for (int k = 0; k < b; ++k) {
    const u64 rk = __shfl(row, k, 64);
    if ((row >> k) & 1ull) row |= rk;
  }
  if (lane < b) {
    out[lane * ldo] = row | (1ull << lane);
    for (i64 w = 1; w < ldo; ++w) out[lane * ldo + w] = 0ull;
  }
}

// Transpose of a bit matrix, 512 input rows x 16 input words (1,024 columns) per workgroup of eight
// waves, staged through LDS so that both sides move whole lines:
//  1. the tile is read row by row (a wave instruction covers 4 rows x 128 bytes) into LDS;
//  2. wave w takes input words 2w and 2w+1; lane l holds rows 64 b + l of a word column (b < 8),
//     each 64 x 64 bit block is turned by lane shuffles, and lane j then holds output row
//     64 cw + j, words 8 rt + b, which go back to LDS (the same buffer, after a barrier);
//  3. the 1,024 output rows x 8 words (64 contiguous bytes each) are written row by row.
constexpr int kTpRows = 512;
constexpr int kTpWords = 16;
constexpr int kTpInLd = kTpWords + 1;  // padded LDS row strides (u64 words)
constexpr int kTpOutLd = 8 + 1;
constexpr int kTpLds = (kTpRows * kTpInLd > 64 * kTpWords * kTpOutLd) ? kTpRows * kTpInLd : 64 * kTpWords * kTpOutLd;

// 64 x 64 bit block held one row per lane (bit j = column j) -> one column per lane, in six
// butterfly stages: at stage s the lanes whose bit s is clear trade their columns with bit s set
// for the partner lane's (lane ^ s) columns with bit s clear.
__device__ __forceinline__ u64 transpose_block64(u64 x) {
  const int lane = threadIdx.x & 63;
  constexpr u64 kLow[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                           0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int s = 32 >> st;
    const u64 lo = kLow[st];
    const u64 y = __shfl_xor(x, s, 64);
    x = (lane & s) ? ((x & ~lo) | ((y & ~lo) >> s)) : ((x & lo) | ((y & lo) << s));
  }
  return x;
}

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4)))  // two workgroups per CU
k_transpose(const u64* __restrict__ in, i64 rows, i64 cols, i64 ldi, u64* __restrict__ out, i64 ldo,
            const u32* __restrict__ pred, u32 pred_val) {
  __shared__ u64 buf[kTpLds];
  if (pred && *pred != pred_val) return;  // the product this transpose feeds does not run
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const i64 rwords = (rows + 63) >> 6, cwords = (cols + 63) >> 6;
  const i64 rtiles = (rows + kTpRows - 1) / kTpRows;
  const i64 tile = blockIdx.x;  // one tile per workgroup
  const i64 rt = tile % rtiles, ct = tile / rtiles;  // row tiles fastest: neighbours share output lines
  // 1. rows of the tile -> LDS (rows past the matrix read as zero, words past it are never used);
  //    32-bit offsets from the tile's first word, clamped into the matrix
  const u64* src = in + rt * kTpRows * ldi + ct * kTpWords;
  const int rlast = (int)(rows - 1 - rt * kTpRows < kTpRows - 1 ? rows - 1 - rt * kTpRows : kTpRows - 1);
  const int clast = (int)(cwords - 1 - ct * kTpWords < kTpWords - 1 ? cwords - 1 - ct * kTpWords : kTpWords - 1);
  u64 v[kTpRows * kTpWords / 512];
#pragma unroll
  for (int i = 0; i < kTpRows * kTpWords / 512; ++i) {
    const int f = t + 512 * i, r = f / kTpWords, c = f % kTpWords;
    v[i] = src[(u32)(r < rlast ? r : rlast) * (u32)ldi + (u32)(c < clast ? c : clast)];
  }
#pragma unroll
  for (int i = 0; i < kTpRows * kTpWords / 512; ++i) {
    const int f = t + 512 * i, r = f / kTpWords, c = f % kTpWords;
    buf[r * kTpInLd + c] = r <= rlast ? v[i] : 0ull;
  }
  __syncthreads();
  // 2. turn the 64 x 64 blocks
  u64 x[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < 8; ++b) x[h][b] = buf[(64 * b + lane) * kTpInLd + 2 * wave + h];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < 8; ++b) x[h][b] = transpose_block64(x[h][b]);
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < 8; ++b) buf[((2 * wave + h) * 64 + lane) * kTpOutLd + b] = x[h][b];
  __syncthreads();
  // 3. output rows 64 ct kTpWords .. , words 8 rt .. 8 rt + 7
  u64* dst = out + ct * (64 * kTpWords) * ldo + rt * 8;
  const i64 olast = cols - 1 - ct * (64 * kTpWords), wlast = rwords - 1 - rt * 8;
#pragma unroll
  for (int i = 0; i < 64 * kTpWords * 8 / 512; ++i) {
    const int f = t + 512 * i, o = f / 8, b = f % 8;
    if (o <= olast && b <= wlast) dst[(u32)o * (u32)ldo + (u32)b] = buf[o * kTpOutLd + b];
  }
}

__global__ void k_check_pad(const u64* __restrict__ a, i64 rows, i64 n, i64 ld, u32* __restrict__ bad) {
  const i64 nw = (n + 63) >> 6;
  const u64 lm = last_word_mask(n);
  const i64 total = rows * ld;
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    const i64 w = t % ld;
    const u64 x = a[t];
    const bool b = (w >= nw) ? (x != 0) : (w == nw - 1 && (x & ~lm) != 0);
    if (b) atomicOr(bad, 1u);
  }
}

__device__ inline int wave_reduce_add(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline int wave_excl_scan(int v, int lane) {
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x - v;
}

// Set bits of one row, summed over the wave (every lane gets the sum).  Each lane reads four words
// per step (lane + 64 j), all four loads issued before any is used: they are clamped into the row
// instead of guarded, and words past it are dropped.
__device__ __forceinline__ u32 wave_row_bits(const u64* __restrict__ row, i64 nw, int lane) {
  u32 c = 0;
  for (i64 w0 = 0; w0 < nw; w0 += 256) {
    u64 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const i64 w = w0 + lane + 64 * j;
      v[j] = row[w < nw ? w : nw - 1];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (w0 + lane + 64 * j < nw) c += (u32)__popcll(v[j]);
  }
  return (u32)wave_reduce_add((int)c);
}

// one wave per row
__global__ void k_row_popcount(const u64* __restrict__ a, i64 rows, i64 n, i64 ld, int32_t* __restrict__ deg,
                               unsigned long long* __restrict__ total) {
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  const i64 nw = (n + 63) >> 6;
  for (i64 row = wave; row < rows; row += nwaves) {
    const u32 c = wave_row_bits(a + row * ld, nw, lane);
    if (lane == 0) {
      deg[row] = (int32_t)c;
      if (total) atomicAdd(total, (unsigned long long)c);
    }
  }
}

// Set bits of four rows r0 + k stride (k < 4; rows past the matrix count 0), summed over the wave: all
// 16 loads of a lane are in flight together.
__device__ __forceinline__ void wave_rows_bits4(const u64* __restrict__ a, i64 ld, i64 nw, i64 rows, i64 r0,
                                                i64 stride, int lane, u32 (&c)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) c[k] = 0;
  for (i64 w0 = 0; w0 < nw; w0 += 256) {
    u64 v[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const i64 r = r0 + k * stride, rc = r < rows ? r : rows - 1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const i64 w = w0 + lane + 64 * j;
        v[k][j] = a[rc * ld + (w < nw ? w : nw - 1)];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (r0 + k * stride < rows && w0 + lane + 64 * j < nw) c[k] += (u32)__popcll(v[k][j]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) c[k] = (u32)wave_reduce_add((int)c[k]);
}

// The two reductions below end in a few global atomics per workgroup on one address each; those
// serialize, so they run on few workgroups (kStatBlocks) whose waves read four rows at a time.
constexpr int kStatBlocks = 256;

// total number of set bits
__global__ void k_popcount_total(const u64* __restrict__ a, i64 rows, i64 nw, i64 ld,
                                 unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[4];
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  unsigned long long tot = 0;
  for (i64 r0 = wave; r0 < rows; r0 += 4 * nwaves) {
    u32 c[4];
    wave_rows_bits4(a, ld, nw, rows, r0, nwaves, lane, c);
    tot += (unsigned long long)c[0] + c[1] + c[2] + c[3];
  }
  if (lane == 0) part[threadIdx.x >> 6] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = part[0] + part[1] + part[2] + part[3];
    if (t) atomicAdd(total, t);
  }
}

// degree statistics of a relation: total, largest row, nonempty rows
__global__ void k_graph_stats(const u64* __restrict__ a, i64 rows, i64 nw, i64 ld, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long s_tot[4], s_max[4], s_ne[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  unsigned long long tot = 0, mx = 0, ne = 0;
  for (i64 r0 = wave; r0 < rows; r0 += 4 * nwaves) {
    u32 c[4];
    wave_rows_bits4(a, ld, nw, rows, r0, nwaves, lane, c);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      tot += c[k];
      mx = c[k] > mx ? c[k] : mx;
      ne += c[k] ? 1u : 0u;
    }
  }
  if (lane == 0) {
    s_tot[wv] = tot;
    s_max[wv] = mx;
    s_ne[wv] = ne;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0, m = 0, e = 0;
    for (int i = 0; i < 4; ++i) {
      t += s_tot[i];
      m = s_max[i] > m ? s_max[i] : m;
      e += s_ne[i];
    }
    if (t) atomicAdd(&out[0], t);
    if (m) atomicMax(&out[1], m);
    if (e) atomicAdd(&out[2], e);
  }
}

// single workgroup exclusive scan: rp[0] = 0, rp[i+1] = rp[i] + deg[i].  Segments of 8,192 degrees:
// each thread sums eight consecutive ones (loads clamped and issued together), the sums are scanned
// by wave shuffles and then across the 16 waves, and the running total carries to the next segment.
constexpr int kScanPer = 8;

__global__ void __launch_bounds__(1024) k_scan_rowptr(const int32_t* __restrict__ deg, i64 n, i64* __restrict__ rp) {
  __shared__ i64 wsum[16];
  __shared__ i64 wpre[17];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  i64 carry = 0;
  for (i64 base = 0; base < n; base += 1024 * kScanPer) {
    int v[kScanPer];
    const i64 i0 = base + (i64)t * kScanPer;
    if (i0 + kScanPer <= n) {
      // eight consecutive degrees as two 16-byte loads (deg is 16-byte aligned, i0 a multiple of 8)
      const int4 a = *(const int4*)(deg + i0), b = *(const int4*)(deg + i0 + 4);
      v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
    } else {
#pragma unroll
      for (int j = 0; j < kScanPer; ++j) {
        const i64 i = i0 + j;
        v[j] = deg[i < n ? i : n - 1];
      }
    }
    i64 sum = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      if (base + (i64)t * kScanPer + j >= n) v[j] = 0;
      sum += v[j];
    }
    i64 x = sum;  // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const i64 y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (t == 0) {
      i64 r = 0;
      for (int w = 0; w < 16; ++w) {
        wpre[w] = r;
        r += wsum[w];
      }
      wpre[16] = r;
    }
    __syncthreads();
    i64 run = carry + wpre[wave] + x - sum;
    i64 out[kScanPer];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      out[j] = run;
      run += v[j];
    }
    if (i0 + kScanPer <= n) {
      // rp is 16-byte aligned and i0 a multiple of 8: four 16-byte stores
#pragma unroll
      for (int j = 0; j < kScanPer; j += 2) *(longlong2*)(rp + i0 + j) = make_longlong2(out[j], out[j + 1]);
    } else {
#pragma unroll
      for (int j = 0; j < kScanPer; ++j)
        if (i0 + j < n) rp[i0 + j] = out[j];
    }
    carry += wpre[16];
    __syncthreads();  // wsum and wpre are rewritten by the next segment
  }
  if (t == 0) rp[n] = carry;
}

// Relabelling of the nodes: dst[i][j] = src[perm[i]][perm[j]] for i, j < n (padding words of dst zero).
// A workgroup takes RPB output rows at a time with their source rows staged in LDS; a wave assembles
// the rows' words w0 .. w0 + 7 together: lane b reads perm[64 w + b] once (whole lines) and tests that
// column in every staged row, one ballot per (row, word), so the permutation is read once per RPB rows.
// The row loops are unrolled so that the loads and LDS reads of a pass are all in flight together.
template <int RPB>
__global__ void __launch_bounds__(256)
k_permute(const u64* __restrict__ src, i64 lds_, const int32_t* __restrict__ perm, i64 n, u64* __restrict__ dst,
          i64 ldd) {
  extern __shared__ u64 srow[];  // RPB x nw
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const i64 nw = (n + 63) >> 6;
  for (i64 i0 = blockIdx.x * (i64)RPB; i0 < n; i0 += (i64)gridDim.x * RPB) {
    const int rows = (int)(n - i0 < RPB ? n - i0 : RPB);
    i64 pis[RPB];
#pragma unroll
    for (int r = 0; r < RPB; ++r) {
      const i64 pi = r < rows ? (i64)perm[i0 + r] : -1;
      pis[r] = (pi >= 0 && pi < n) ? pi : -1;
    }
    for (i64 w = threadIdx.x; w < nw; w += 256) {
      u64 v[RPB];
#pragma unroll
      for (int r = 0; r < RPB; ++r) v[r] = pis[r] >= 0 ? src[pis[r] * lds_ + w] : 0ull;
#pragma unroll
      for (int r = 0; r < RPB; ++r) srow[(i64)r * nw + w] = v[r];
    }
    __syncthreads();
    for (i64 w0 = wv * 8; w0 < ldd; w0 += 32) {
      int32_t cs[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const i64 j = (w0 + q) * 64 + lane;
        const int32_t c = (w0 + q < nw && j < n) ? perm[j] : -1;
        cs[q] = (c >= 0 && c < n) ? c : -1;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t c = cs[q];
        const i64 cw = c >= 0 ? (c >> 6) : 0;
        const int cb = c & 63;
        u64 x[RPB];
#pragma unroll
        for (int r = 0; r < RPB; ++r) x[r] = srow[(i64)r * nw + cw];  // rows past `rows` hold stale data
        u64 keep = 0ull;  // lane r keeps row r's word
#pragma unroll
        for (int r = 0; r < RPB; ++r) {
          const u64 v = __ballot(c >= 0 && ((x[r] >> cb) & 1ull));
          if (lane == r) keep = v;
        }
        if (lane < rows && w0 + q < ldd) dst[(i0 + lane) * ldd + w0 + q] = keep;
      }
    }
    __syncthreads();
  }
}

// CSC (in-edges) from a CSR: in-degrees counted with atomics, then each edge (u, v) placed in v's
// segment at a slot taken from v's cursor.  The order inside a segment is whichever the atomics give.
__global__ void k_csc_count(const int32_t* __restrict__ ci, i64 m, int32_t* __restrict__ degt) {
  for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x)
    atomicAdd(&degt[ci[e]], 1);
}

__global__ void k_csc_fill(const i64* __restrict__ rp, const int32_t* __restrict__ ci, i64 n, i64 m,
                           const i64* __restrict__ rpt, int32_t* __restrict__ cursor, int32_t* __restrict__ cit) {
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  for (i64 u = wave; u < n; u += nwaves) {
    const i64 e1 = rp[u + 1];
    for (i64 e = rp[u] + lane; e < e1; e += 64) {
      const int32_t v = ci[e];
      const i64 pos = rpt[v] + atomicAdd(&cursor[v], 1);
      if (pos < m) cit[pos] = (int32_t)u;  // always: the CSR holds m edges
    }
  }
}

// one wave per row; lanes own consecutive words
__global__ void k_bits_to_csr(const u64* __restrict__ a, i64 rows, i64 n, i64 ld, const i64* __restrict__ rp,
                              int32_t* __restrict__ ci) {
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  const i64 nw = (n + 63) >> 6;
  for (i64 row = wave; row < rows; row += nwaves) {
    i64 base = rp[row];
    for (i64 w0 = 0; w0 < nw; w0 += 64) {
      const i64 w = w0 + lane;
      u64 x = (w < nw) ? a[row * ld + w] : 0ull;
      const int pc = __popcll(x);
      const int ex = wave_excl_scan(pc, lane);
      const int tot = __shfl(ex + pc, 63, 64);
      i64 pos = base + ex;
      while (x) {
        const int b = __ffsll((unsigned long long)x) - 1;
        ci[pos++] = (int32_t)(w * 64 + b);
        x &= x - 1;
      }
      base += tot;
    }
  }
}

}  // namespace

hipError_t launch_fill_random(u64* a, i64 rows, i64 n, i64 ld, u64 seed, int s_in, int s_out, i64 brows, i64 bwords,
                              hipStream_t s) {
  if (rows <= 0 || ld <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_random, dim3(grid_for(rows * ld, kBlock, 16384)), dim3(kBlock), 0, s, a, rows, n, ld, seed,
                     s_in, s_out, brows, bwords);
  return hipGetLastError();
}

hipError_t launch_fill_zero(u64* p, i64 nwords, hipStream_t s) {
  if (nwords <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(nwords, kBlock, 16384)), dim3(kBlock), 0, s, p, nwords);
  return hipGetLastError();
}

hipError_t launch_pack_u8(const uint8_t* d, i64 rows, i64 n, i64 ldd, u64* bits, i64 ld, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_u8, dim3(grid_for(rows * ld * 64, kBlock, 16384)), dim3(kBlock), 0, s, d, rows, n, ldd,
                     bits, ld);
  return hipGetLastError();
}

hipError_t launch_unpack_u8(const u64* bits, i64 rows, i64 n, i64 ld, uint8_t* d, i64 ldd, hipStream_t s) {
  if (rows <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_u8, dim3(grid_for(rows * n, kBlock, 16384)), dim3(kBlock), 0, s, bits, rows, n, ld, d,
                     ldd);
  return hipGetLastError();
}

hipError_t launch_pack_coo(const int32_t* r, const int32_t* c, i64 m, i64 rows, i64 n, u64* bits, i64 ld, u32* bad,
                           hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_coo, dim3(grid_for(m, kBlock, 16384)), dim3(kBlock), 0, s, r, c, m, rows, n, bits, ld,
                     bad);
  return hipGetLastError();
}

hipError_t launch_ewise(int op, const u64* a, i64 lda, const u64* b, i64 ldb, u64* c, i64 ldc, i64 rows, i64 n,
                        hipStream_t s, const u32* pred, u32 pred_val) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ewise, dim3(grid_for(rows * ldc, kBlock, 16384)), dim3(kBlock), 0, s, op, a, lda, b, ldb, c,
                     ldc, rows, n, pred, pred_val);
  return hipGetLastError();
}

hipError_t launch_zero_pad(u64* a, i64 rows, i64 n, i64 ld, hipStream_t s) {
  const i64 nw = words_for(n);
  if (rows <= 0 || ld <= nw) return hipSuccess;
  hipLaunchKernelGGL(k_zero_pad, dim3(grid_for(rows * (ld - nw), kBlock, 16384)), dim3(kBlock), 0, s, a, rows, nw, ld);
  return hipGetLastError();
}

hipError_t launch_set_diag(u64* a, i64 ld, i64 rows, i64 n, hipStream_t s) {
  const i64 cnt = rows < n ? rows : n;
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_diag, dim3(grid_for(cnt)), dim3(kBlock), 0, s, a, ld, cnt);
  return hipGetLastError();
}

hipError_t launch_set_onehot(u64* a, i64 ld, const int32_t* idx, i64 k, i64 n, u32* bad, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_onehot, dim3(grid_for(k)), dim3(kBlock), 0, s, a, ld, idx, k, n, bad);
  return hipGetLastError();
}

hipError_t launch_rows_by_index(const u64* C, i64 ldc, const int32_t* idx, i64 k, i64 n, int reflexive, u64* out,
                               i64 ldo, u32* bad, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (ldo <= 0) return hipSuccess;
  const i64 blocks = k * ((ldo + kRowSegWords - 1) / kRowSegWords);
  hipLaunchKernelGGL(k_rows_by_index, dim3((unsigned)std::min<i64>(blocks, 1 << 20)), dim3(kBlock), 0, s, C, ldc, idx,
                     k, n, reflexive, out, ldo, bad);
  return hipGetLastError();
}

hipError_t launch_closure64(const u64* M, i64 ldm, i64 b, u64* out, i64 ldo, hipStream_t s) {
  if (b <= 0) return hipSuccess;
  if (b > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_closure64, dim3(1), dim3(64), 0, s, M, ldm, b, out, ldo);
  return hipGetLastError();
}

hipError_t launch_rows_from_rp(const i64* rp, i64 rows, int32_t* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_from_rp, dim3(grid_for(rows * 64, kBlock, 16384)), dim3(kBlock), 0, s, rp, rows, out);
  return hipGetLastError();
}

hipError_t launch_nonempty_rows(const u64* a, i64 rows, i64 n, i64 ld, int32_t* list, u32* count, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nonempty_rows, dim3(grid_for(rows * 8, kBlock, 16384)), dim3(kBlock), 0, s, a, rows,
                     words_for(n), ld, list, count);
  return hipGetLastError();
}

hipError_t launch_copy_rows(const u64* src, i64 lds, const int32_t* list, i64 k, i64 n, u64* dst, i64 ldd,
                            hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_rows, dim3(grid_for(k * 64, kBlock, 16384)), dim3(kBlock), 0, s, src, lds, list, k,
                     words_for(n), dst, ldd);
  return hipGetLastError();
}

hipError_t launch_check_index(const int32_t* idx, i64 k, i64 n, u32* bad, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_index, dim3(grid_for(k)), dim3(kBlock), 0, s, idx, k, n, bad);
  return hipGetLastError();
}

i64 gather_cols_max_n() { return (i64)64 * 8192; }  // the staged row: 64 KiB of LDS

hipError_t launch_gather_cols(const u64* T, i64 ldt, i64 rows, i64 n, const int32_t* cols, i64 b, int diag, u64* A,
                              i64 lda, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (n > gather_cols_max_n() || n <= 0) return hipErrorInvalidValue;
  const size_t lds = (size_t)words_for(n) * sizeof(u64);
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)(rows < 65535 ? rows : 65535)), dim3(256), lds, s, T, ldt, rows, n,
                     cols, b, diag, A, lda);
  return hipGetLastError();
}

hipError_t launch_transpose(const u64* in, i64 rows, i64 cols, i64 ldi, u64* out, i64 ldo, hipStream_t s,
                            const u32* pred, u32 pred_val) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const i64 nwo = words_for(rows);
  if (ldo > nwo && !pred) {
    hipError_t e = launch_fill_zero(out, cols * ldo, s);
    if (e != hipSuccess) return e;
  }
  // the kernel addresses a tile with 32-bit offsets
  if ((i64)kTpRows * ldi >= (1ll << 32) || (i64)64 * kTpWords * ldo >= (1ll << 32)) return hipErrorInvalidValue;
  const i64 tiles = ((rows + kTpRows - 1) / kTpRows) * ((words_for(cols) + kTpWords - 1) / kTpWords);
  if (tiles >= (1ll << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)tiles), dim3(512), 0, s, in, rows, cols, ldi, out, ldo, pred,
                     pred_val);
  return hipGetLastError();
}

hipError_t launch_check_pad(const u64* a, i64 rows, i64 n, i64 ld, u32* bad, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_pad, dim3(grid_for(rows * ld, kBlock, 16384)), dim3(kBlock), 0, s, a, rows, n, ld, bad);
  return hipGetLastError();
}

hipError_t launch_row_popcount(const u64* a, i64 rows, i64 n, i64 ld, int32_t* deg, unsigned long long* total,
                               hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_popcount, dim3(grid_for(rows * 64, kBlock, 16384)), dim3(kBlock), 0, s, a, rows, n, ld, deg,
                     total);
  return hipGetLastError();
}

hipError_t launch_popcount_total(const u64* a, i64 rows, i64 n, i64 ld, unsigned long long* total, hipStream_t s) {
  if (rows <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_popcount_total, dim3(grid_for(rows * 64, kBlock, kStatBlocks)), dim3(kBlock), 0, s, a, rows,
                     words_for(n), ld, total);
  return hipGetLastError();
}

// (set bits, largest row count, nonempty rows) from per-row counts, by one workgroup with plain stores into
// out[0..2] (no atomics, nothing to clear first)
__global__ void __launch_bounds__(1024) k_deg_stats(const int32_t* __restrict__ deg, i64 n,
                                                    unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[16][3];
  unsigned long long sum = 0, mx = 0, ne = 0;
#pragma unroll 8
  for (i64 i = threadIdx.x; i < n; i += 1024) {
    const unsigned long long d = (unsigned long long)deg[i];
    sum += d;
    mx = d > mx ? d : mx;
    ne += d != 0ull ? 1ull : 0ull;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off, 64);
    const unsigned long long m2 = __shfl_xor(mx, off, 64);
    mx = m2 > mx ? m2 : mx;
    ne += __shfl_xor(ne, off, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[wv][0] = sum;
    part[wv][1] = mx;
    part[wv][2] = ne;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      s0 += part[w][0];
      s1 = part[w][1] > s1 ? part[w][1] : s1;
      s2 += part[w][2];
    }
    out[0] = s0;
    out[1] = s1;
    out[2] = s2;
  }
}

// The relabelling's classes, from a relation's row and column counts rp, cp (n each), by one workgroup.
// With the largest counts rmax, cmax: a node is heavy as a row when 4 rp >= rmax, as a column when
// 4 cp >= cmax, dead as a row when 64 rp < rmax, as a column when 64 cp < cmax.  out (9 u64): rmax, cmax,
// heavy rows, heavy columns, dead nodes (dead row or column), 256-node tiles holding a dead row, tiles
// holding a dead column, and two zero words.  Tiles are flagged in LDS: n <= 256 * kRelabelTiles.
constexpr int kRelabelTiles = 1024;
__device__ __forceinline__ unsigned long long block_sum_1024(unsigned long long v, unsigned long long* part) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();  // part may still be read by a previous call
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long t = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) t += part[w];
  return t;
}
__device__ __forceinline__ unsigned long long block_max_1024(unsigned long long v, unsigned long long* part) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long t = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) t = part[w] > t ? part[w] : t;
  return t;
}

__global__ void __launch_bounds__(1024) k_relabel_classes(const int32_t* __restrict__ rp, const int32_t* __restrict__ cp,
                                                          i64 n, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[16];
  __shared__ u32 rt[kRelabelTiles], ct[kRelabelTiles];
  const int t = threadIdx.x;
  const i64 tiles = (n + 255) / 256;
  for (i64 i = t; i < tiles; i += 1024) rt[i] = ct[i] = 0u;
  unsigned long long mr = 0, mc = 0;
  for (i64 v = t; v < n; v += 1024) {
    const unsigned long long a = (unsigned long long)rp[v], b = (unsigned long long)cp[v];
    mr = a > mr ? a : mr;
    mc = b > mc ? b : mc;
  }
  const unsigned long long rmax = block_max_1024(mr, part);
  const unsigned long long cmax = block_max_1024(mc, part);
  unsigned long long hin = 0, hout = 0, dead = 0;
  for (i64 v = t; v < n; v += 1024) {
    const unsigned long long a = (unsigned long long)rp[v], b = (unsigned long long)cp[v];
    hin += 4 * a >= rmax ? 1u : 0u;
    hout += 4 * b >= cmax ? 1u : 0u;
    const bool dr = 64 * a < rmax, dc = 64 * b < cmax;
    dead += (dr || dc) ? 1u : 0u;
    if (dr) rt[v / 256] = 1u;  // benign races: every writer stores 1
    if (dc) ct[v / 256] = 1u;
  }
  hin = block_sum_1024(hin, part);
  hout = block_sum_1024(hout, part);
  dead = block_sum_1024(dead, part);  // its barriers also order the tile flags before they are read
  unsigned long long drt = 0, dct = 0;
  for (i64 i = t; i < tiles; i += 1024) {
    drt += rt[i];
    dct += ct[i];
  }
  drt = block_sum_1024(drt, part);
  dct = block_sum_1024(dct, part);
  if (t == 0) {
    out[0] = rmax;
    out[1] = cmax;
    out[2] = hin;
    out[3] = hout;
    out[4] = dead;
    out[5] = drt;
    out[6] = dct;
    out[7] = 0ull;
    out[8] = 0ull;
  }
}

// The relabelling itself: the nodes ordered by class, in their given order within a class, as perm[new] =
// old and inv[old] = new, by one workgroup (a stable counting sort: thread t takes the nodes of one
// contiguous chunk, a workgroup scan gives each thread its place in every class).  mode 1: the four
// heavy/light classes (0 heavy row and light column, 1 heavy both, 2 light row and heavy column, 3 light
// both); mode 2: the dead nodes after all others.  rmax, cmax are k_relabel_classes' out[0], out[1].
__global__ void __launch_bounds__(1024) k_relabel_perm(const int32_t* __restrict__ rp, const int32_t* __restrict__ cp,
                                                       i64 n, int mode, const unsigned long long* __restrict__ maxes,
                                                       int32_t* __restrict__ perm, int32_t* __restrict__ inv) {
  __shared__ unsigned long long wsum[2][16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const unsigned long long rmax = maxes[0], cmax = maxes[1];
  auto cls_of = [&](i64 v) -> int {
    const unsigned long long a = (unsigned long long)rp[v], b = (unsigned long long)cp[v];
    if (mode == 1) {
      const int in = 4 * a >= rmax, out = 4 * b >= cmax;
      return 2 * (1 - in) + (in == out);
    }
    return (64 * a < rmax || 64 * b < cmax) ? 3 : 1;
  };
  const i64 chunk = (n + 1023) / 1024;
  const i64 v0 = (i64)t * chunk, v1 = v0 + chunk < n ? v0 + chunk : n;
  // this thread's count per class, two classes per 64-bit word (32-bit fields: n < 2^31)
  unsigned long long c01 = 0, c23 = 0;
  for (i64 v = v0; v < v1; ++v) {
    const int k = cls_of(v);
    c01 += k == 0 ? 1ull : k == 1 ? (1ull << 32) : 0ull;
    c23 += k == 2 ? 1ull : k == 3 ? (1ull << 32) : 0ull;
  }
  // exclusive scan over the threads: within the wave by shuffles, then over the 16 waves' totals
  unsigned long long s01 = c01, s23 = c23;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long a = __shfl_up(s01, off, 64), b = __shfl_up(s23, off, 64);
    if (lane >= off) {
      s01 += a;
      s23 += b;
    }
  }
  if (lane == 63) {
    wsum[0][wv] = s01;
    wsum[1][wv] = s23;
  }
  __syncthreads();
  unsigned long long b01 = 0, b23 = 0, t01 = 0, t23 = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    if (w < wv) {
      b01 += wsum[0][w];
      b23 += wsum[1][w];
    }
    t01 += wsum[0][w];
    t23 += wsum[1][w];
  }
  s01 += b01 - c01;  // exclusive prefix of this thread
  s23 += b23 - c23;
  // the first position of each class, then of this thread within it
  const i64 tot0 = (i64)(t01 & 0xFFFFFFFFull), tot1 = (i64)(t01 >> 32), tot2 = (i64)(t23 & 0xFFFFFFFFull);
  i64 pos[4] = {(i64)(s01 & 0xFFFFFFFFull), tot0 + (i64)(s01 >> 32), tot0 + tot1 + (i64)(s23 & 0xFFFFFFFFull),
                tot0 + tot1 + tot2 + (i64)(s23 >> 32)};
  for (i64 v = v0; v < v1; ++v) {
    const int k = cls_of(v);
    const i64 p = pos[k]++;
    perm[p] = (int32_t)v;
    inv[v] = (int32_t)p;
  }
}

hipError_t launch_relabel_classes(const int32_t* rp, const int32_t* cp, i64 n, unsigned long long* out, hipStream_t s) {
  if (n <= 0 || (n + 255) / 256 > kRelabelTiles) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_relabel_classes, dim3(1), dim3(1024), 0, s, rp, cp, n, out);
  return hipGetLastError();
}

hipError_t launch_relabel_perm(const int32_t* rp, const int32_t* cp, i64 n, int mode, const unsigned long long* maxes,
                               int32_t* perm, int32_t* inv, hipStream_t s) {
  if (n <= 0 || (mode != 1 && mode != 2)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_relabel_perm, dim3(1), dim3(1024), 0, s, rp, cp, n, mode, maxes, perm, inv);
  return hipGetLastError();
}

hipError_t launch_deg_stats(const int32_t* deg, i64 n, unsigned long long* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_deg_stats, dim3(1), dim3(1024), 0, s, deg, n, out);
  return hipGetLastError();
}

hipError_t launch_graph_stats(const u64* a, i64 rows, i64 n, i64 ld, unsigned long long* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_stats, dim3(grid_for(rows * 64, kBlock, kStatBlocks)), dim3(kBlock), 0, s, a, rows,
                     words_for(n), ld, out);
  return hipGetLastError();
}

hipError_t launch_scan_rowptr(const int32_t* deg, i64 n, i64* rp, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_rowptr, dim3(1), dim3(1024), 0, s, deg, n, rp);
  return hipGetLastError();
}

hipError_t launch_permute(const u64* src, i64 lds_, const int32_t* perm, i64 n, u64* dst, i64 ldd, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const i64 nw = words_for(n);
  const size_t row_bytes = (size_t)nw * sizeof(u64);
  if (row_bytes > 64 * 1024) return hipErrorInvalidValue;
  // staged rows: 16 while they fit in 32 KB of LDS, else 4 (n <= 65,536), else 1
  auto go = [&](auto rpb_tag) {
    constexpr int RPB = decltype(rpb_tag)::value;
    const i64 blocks = (n + RPB - 1) / RPB;
    hipLaunchKernelGGL(k_permute<RPB>, dim3((unsigned)(blocks < 65535 ? blocks : 65535)), dim3(256), row_bytes * RPB,
                       s, src, lds_, perm, n, dst, ldd);
  };
  if (row_bytes * 16 <= 32 * 1024) go(std::integral_constant<int, 16>{});
  else if (row_bytes * 4 <= 32 * 1024) go(std::integral_constant<int, 4>{});
  else go(std::integral_constant<int, 1>{});
  return hipGetLastError();
}

hipError_t launch_csc_from_csr(const i64* rp, const int32_t* ci, i64 n, i64 m, int32_t* degt, int32_t* cursor,
                               i64* rpt, int32_t* cit, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipError_t e = launch_fill_zero((u64*)degt, (n + 1) / 2, s);
  if (e == hipSuccess) e = launch_fill_zero((u64*)cursor, (n + 1) / 2, s);
  if (e != hipSuccess) return e;
  if (m > 0) {
    hipLaunchKernelGGL(k_csc_count, dim3(grid_for(m, kBlock, 16384)), dim3(kBlock), 0, s, ci, m, degt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_scan_rowptr(degt, n, rpt, s)) != hipSuccess) return e;
  if (m > 0) {
    hipLaunchKernelGGL(k_csc_fill, dim3(grid_for(n * 64, kBlock, 16384)), dim3(kBlock), 0, s, rp, ci, n, m, rpt,
                       cursor, cit);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_bits_to_csr(const u64* a, i64 rows, i64 n, i64 ld, const i64* rp, int32_t* ci, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bits_to_csr, dim3(grid_for(rows * 64, kBlock, 16384)), dim3(kBlock), 0, s, a, rows, n, ld, rp,
                     ci);
  return hipGetLastError();
}

}  // namespace bmlp
