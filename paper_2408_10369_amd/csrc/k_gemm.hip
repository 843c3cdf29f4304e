// Boolean-semiring matrix product with OR-accumulate:
//     C = Cold | A.B,   (A.B)_ij = OR_k (A_ik AND B_kj)      (Section 2)
// plus the semi-naive delta D = C & ~Cold and a wave-ballot "changed" flag
// (the fixpoint test of Algorithms 1 and 2: iterates only grow, so "some word
// changed" is the same test as "the matrices differ").
//
// VALU arm (bit-packed).  Row-OR formulation: C[i,:] |= B[k,:] for every set
// bit A[i,k].  A workgroup owns a tile of TR rows x TW words of C.  Each wave
// owns RPW rows; each lane owns WPL words of those rows.  For every chunk of
// 64 k values the workgroup stages B[k0..k0+63, tile words] in LDS; the A word
// of each of the wave's rows is wave-uniform, so the AND mask for (i, k) is a
// scalar value and every lane does one v_and_or per 32 bit-MACs.  Chunks in
// which no row of the tile has a set A bit are skipped entirely (sparse A).
//
// Split-K.  When the output has too few tiles to fill the chip, the k range
// is split over several workgroups and partial results are merged with 64-bit
// atomic ORs.  OR is idempotent and commutative, so the merge is exact.  C is
// first made equal to Cold; a bit is new exactly when the atomic that sets it
// returns an old word without it, which gives D and the changed flag exactly.
#include "bmlp_internal.h"
#include "valu_tile.h"

namespace bmlp {

namespace {

template <int RPW, int WPL>
__global__ void __launch_bounds__(256)
k_gemm_valu(const u64* __restrict__ A, i64 lda, const u64* __restrict__ B, i64 ldb, const u64* __restrict__ Cold,
            i64 ldco, u64* __restrict__ C, i64 ldc, u64* __restrict__ D, i64 ldd, i64 M, i64 K, i64 N,
            u32* __restrict__ changed, int ksplit, int chunks_per_split, unsigned long long* __restrict__ newbits,
            const u32* __restrict__ pred, u32 pred_val) {
  constexpr int TW = 64 * WPL;
  constexpr int TR = 4 * RPW;
  __shared__ u64 Bs[64][TW];
  if (pred && *pred != pred_val) return;  // another arm serves this round
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const i64 nw = (N + 63) >> 6;
  const i64 ctiles = (nw + TW - 1) / TW;
  const i64 rtiles = (M + TR - 1) / TR;
  // block order: row tiles fastest, then column tiles, then k splits, so that
  // concurrently running workgroups share the B chunks they stage
  const i64 tile = blockIdx.x;
  const i64 rt = tile % rtiles;
  const i64 ct = (tile / rtiles) % ctiles;
  const i64 ks = tile / (rtiles * ctiles);
  const i64 row0 = rt * TR + (i64)wave * RPW;
  const i64 w0 = ct * TW;

  u32 acc[RPW][WPL][2];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int wl = 0; wl < WPL; ++wl) acc[r][wl][0] = acc[r][wl][1] = 0u;

  const i64 kwords = (K + 63) >> 6;
  const i64 kw_begin = ks * chunks_per_split;
  const i64 kw_end = (kw_begin + chunks_per_split < kwords) ? kw_begin + chunks_per_split : kwords;
  valu_tile_accumulate<RPW, WPL>(A, lda, B, ldb, M, K, nw, row0, w0, kw_begin, kw_end, Bs, acc);

  int ch = 0;
  u32 pop = 0;
  if (ksplit == 1) {
    ch = valu_tile_store<RPW, WPL>(acc, Cold, ldco, C, ldc, D, ldd, M, nw, row0, w0, &pop);
  } else {
    // C already holds Cold and D is zero (the launcher sees to both)
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const i64 row = row0 + r;
      if (row >= M) break;
#pragma unroll
      for (int wl = 0; wl < WPL; ++wl) {
        const i64 w = w0 + lane + 64 * wl;
        const u64 v = ((u64)acc[r][wl][1] << 32) | (u64)acc[r][wl][0];
        if (w < nw && v) {
          const u64 old = atomicOr((unsigned long long*)&C[row * ldc + w], (unsigned long long)v);
          const u64 nb = v & ~old;
          if (nb) {
            if (D) atomicOr((unsigned long long*)&D[row * ldd + w], (unsigned long long)nb);
            ch = 1;
            pop += (u32)__popcll(nb);
          }
        }
      }
    }
  }
  wave_count(pop, newbits);
  if (changed) {
    const u64 bal = __ballot(ch);
    if (bal && lane == 0) atomicOr(changed, 1u);
  }
}

template <int RPW>
hipError_t launch_rpw(const GemmArgs& g, hipStream_t s, i64 target_blocks) {
  constexpr int WPL = 1;
  const i64 nw = words_for(g.N);
  const i64 ctiles = (nw + 64 * WPL - 1) / (64 * WPL);
  const i64 rtiles = (g.M + 4 * RPW - 1) / (4 * RPW);
  const i64 kwords = words_for(g.K);
  const i64 tiles = ctiles * rtiles;
  i64 ksplit = 1;
  if (tiles < target_blocks && kwords > 1) {
    ksplit = (target_blocks + tiles - 1) / tiles;
    if (ksplit > kwords) ksplit = kwords;
  }
  i64 cps = (kwords + ksplit - 1) / ksplit;
  if (cps < 1) cps = 1;
  ksplit = (kwords + cps - 1) / cps;
  if (ksplit < 1) ksplit = 1;
  if (ksplit > 1) {
    // C := Cold (unless C is Cold), D := 0
    if (g.Cold && g.Cold != g.C) {
      hipError_t e = launch_ewise(4, g.Cold, g.ldco, nullptr, 0, g.C, g.ldc, g.M, g.N, s);
      if (e != hipSuccess) return e;
    } else if (!g.Cold) {
      hipError_t e = launch_ewise(4, g.C, g.ldc, nullptr, 0, g.C, g.ldc, g.M, 0, s);  // zero C rows
      if (e != hipSuccess) return e;
    }
    if (g.D) {
      hipError_t e = launch_ewise(4, g.D, g.ldd, nullptr, 0, g.D, g.ldd, g.M, 0, s);  // zero D rows
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL((k_gemm_valu<RPW, WPL>), dim3((unsigned)(tiles * ksplit)), dim3(256), 0, s, g.A, g.lda, g.B,
                     g.ldb, g.Cold, g.ldco, g.C, g.ldc, g.D, g.ldd, g.M, g.K, g.N, g.changed, (int)ksplit, (int)cps,
                     g.newbits, g.pred, g.pred_val);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MFMA arm: int8 matrix cores, int32 accumulation, "> 0" threshold.
//
// The operands stay bit-packed in memory; each lane expands the bits it feeds
// to one v_mfma_i32_16x16x64_i8 into 16 bytes with one AND per dword: dword
// (h, j) = (half h of the 64-bit word) & (0x01010101 << j) keeps bits j, j+8,
// j+16, j+24 of that half in place, so byte b holds 0 or 2^j.  Lane group
// g = lane / 16 takes j in {g, g+4} of both halves, so the four groups cover
// all 64 bits.  A and B use the same bit -> (lane group, byte, value) map, so
// every product term is 0 or (+-2^j)^2 = 4^j > 0 (the byte 2^7 reads as -128,
// whose square is positive), and the int32 sum is positive exactly when some
// k has A_ik = B_kj = 1: the OR of ANDs.  The sum per 64-bit word of k is at
// most 8 * (4^0 + ... + 4^7) = 174,760, so it stays exact below 2^31 for up to
// kMaxKWords words of k.  A sum does not depend on the order of its terms, so
// the result is exact whatever k order the instruction assigns to (group,
// byte) -- it only has to be the same for both operands.  B is consumed
// transposed (B^T rows = columns of B), so that a column's 64 k-bits are one
// word, like a row of A.
//
// Tile: a workgroup of 8 waves (two per SIMD, so that one wave's expansion and
// LDS reads overlap the other's matrix-core work) owns 256 x 256 outputs; wave
// (wr, wc) owns rows 128 wr .. +128 and columns 64 wc .. +64 = 8 x 4 MFMA blocks
// of 16 x 16.  Per chunk of kMChunk words of k the workgroup stages 256 rows of
// A (threads 0..255) and 256 rows of B^T (threads 256..511) in LDS,
// double-buffered: the next chunk is loaded into registers while the current
// one is consumed, so one barrier per chunk suffices.  While staging, the A
// waves also record which words of the chunk are nonzero in any of their rows;
// a consuming wave skips the words of k where all 128 of its rows are zero (a
// wave-uniform test on that mask, which keeps the LDS reads of the next word in
// flight).
// A 16 x 16 int32 block sits in lane l as rows 4*(l/16)+v, column l%16
// (v = 0..3), so a ballot of "acc[v] > 0" holds, in bits 16g..16g+15, the 16
// output bits of row 4g+v.
typedef int v4i_t __attribute__((ext_vector_type(4)));

constexpr int kMT = 256;     // workgroup tile (rows and columns)
constexpr int kMChunk = 8;   // words of k per LDS stage
constexpr int kMPad = 9;     // padded LDS row stride in words (no bank conflicts)
constexpr i64 kMaxKWords = 12288;  // 12,288 * 174,760 < 2^31

__device__ __forceinline__ v4i_t expand_frag(u64 w, u32 m0, u32 m1) {
  const u32 lo = (u32)w, hi = (u32)(w >> 32);
  v4i_t f;
  f.x = (int)(lo & m0);
  f.y = (int)(lo & m1);
  f.z = (int)(hi & m0);
  f.w = (int)(hi & m1);
  return f;
}

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_mfma(const u64* __restrict__ A, i64 lda, const u64* __restrict__ BT, i64 ldbt, const u64* __restrict__ Cold,
            i64 ldco, u64* __restrict__ C, i64 ldc, u64* __restrict__ D, i64 ldd, i64 M, i64 K, i64 N,
            u32* __restrict__ changed, unsigned long long* __restrict__ newbits, const u32* __restrict__ pred,
            u32 pred_val) {
  __shared__ u64 As[2][kMT * kMPad];
  __shared__ u64 Bs[2][kMT * kMPad];
  __shared__ u64 bal[8][16];
  __shared__ u32 zmask[2][4];  // per stage and A-staging wave: bit q = some row has a nonzero word q
  if (pred && *pred != pred_val) return;  // another arm serves this round
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;  // wave owns rows wr*128 .. +128, columns wc*64 .. +64
  const int g = lane >> 4, l16 = lane & 15;
  const u32 m0 = 0x01010101u << g, m1 = 0x10101010u << g;
  const i64 ctiles = (N + kMT - 1) / kMT;
  const i64 tr = blockIdx.x / ctiles, tc = blockIdx.x % ctiles;
  const i64 row0 = tr * kMT, col0 = tc * kMT;
  const i64 kwords = (K + 63) >> 6;

  v4i_t acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4i_t{0, 0, 0, 0};

  // threads 0..255 stage row t of the A tile, threads 256..511 row t-256 of the B^T tile
  const bool isa = t < 256;
  const int tt = t & 255;
  const i64 rr = (isa ? row0 : col0) + tt;
  const bool vr = rr < (isa ? M : N);
  const u64* pr = isa ? A + (vr ? rr : 0) * lda : BT + (vr ? rr : 0) * ldbt;
  u64* stage0 = isa ? &As[0][tt * kMPad] : &Bs[0][tt * kMPad];
  u64* stage1 = isa ? &As[1][tt * kMPad] : &Bs[1][tt * kMPad];
  u64 sr[kMChunk];
#pragma unroll
  for (int q = 0; q < kMChunk; ++q) sr[q] = (vr && q < kwords) ? pr[q] : 0ull;
  int buf = 0;
  for (i64 kc = 0; kc < kwords; kc += kMChunk, buf ^= 1) {
    u64* st = buf ? stage1 : stage0;
#pragma unroll
    for (int q = 0; q < kMChunk; ++q) st[q] = sr[q];
    if (isa) {
      u32 zm = 0;
#pragma unroll
      for (int q = 0; q < kMChunk; ++q) zm |= (__ballot(sr[q] != 0ull) != 0ull ? 1u : 0u) << q;
      if (lane == 0) zmask[buf][wave] = zm;
    }
    __syncthreads();
    const i64 kn = kc + kMChunk;
    if (kn < kwords) {
#pragma unroll
      for (int q = 0; q < kMChunk; ++q) sr[q] = (vr && kn + q < kwords) ? pr[kn + q] : 0ull;
    }
    const u64* as = &As[buf][(wr * 128 + l16) * kMPad];
    const u64* bs = &Bs[buf][(wc * 64 + l16) * kMPad];
    // rows of this wave with a nonzero word q of k (wave-uniform)
    const u32 mask = __builtin_amdgcn_readfirstlane(zmask[buf][2 * wr] | zmask[buf][2 * wr + 1]);
    u64 aw[8], bw[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) aw[i] = as[i * 16 * kMPad];
#pragma unroll
    for (int j = 0; j < 4; ++j) bw[j] = bs[j * 16 * kMPad];
#pragma unroll
    for (int q = 0; q < kMChunk; ++q) {
      u64 an[8], bn[4];
      if (q + 1 < kMChunk) {
#pragma unroll
        for (int i = 0; i < 8; ++i) an[i] = as[i * 16 * kMPad + q + 1];
#pragma unroll
        for (int j = 0; j < 4; ++j) bn[j] = bs[j * 16 * kMPad + q + 1];
      }
      if ((mask >> q) & 1u) {
        v4i_t bf[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = expand_frag(bw[j], m0, m1);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const v4i_t af = expand_frag(aw[i], m0, m1);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[j], acc[i][j], 0, 0, 0);
        }
      }
      if (q + 1 < kMChunk) {
#pragma unroll
        for (int i = 0; i < 8; ++i) aw[i] = an[i];
#pragma unroll
        for (int j = 0; j < 4; ++j) bw[j] = bn[j];
      }
    }
  }

  // epilogue: per block row, ballot "> 0", assemble 16 rows x 1 word, OR with Cold
  const i64 nw = (N + 63) >> 6;
  int ch = 0;
  u32 pop = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const u64 b0 = __ballot(acc[i][j].x > 0);
      const u64 b1 = __ballot(acc[i][j].y > 0);
      const u64 b2 = __ballot(acc[i][j].z > 0);
      const u64 b3 = __ballot(acc[i][j].w > 0);
      if (lane == 0) {
        bal[wave][j * 4 + 0] = b0;
        bal[wave][j * 4 + 1] = b1;
        bal[wave][j * 4 + 2] = b2;
        bal[wave][j * 4 + 3] = b3;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (lane < 16) {
      const int r = lane;  // r = 4 * gg + v
      const int v = r & 3, gg = r >> 2;
      u64 word = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const u64 b = bal[wave][q * 4 + v];
        word |= ((b >> (16 * gg)) & 0xFFFFull) << (16 * q);
      }
      const i64 row = row0 + wr * 128 + i * 16 + r;
      const i64 w = (col0 + wc * 64) / 64;
      if (row < M && w < nw) {
        const u64 old = Cold ? Cold[row * ldco + w] : 0ull;
        const u64 nv = word | old;
        C[row * ldc + w] = nv;
        if (D) D[row * ldd + w] = nv & ~old;
        ch |= (nv != old);
        pop += (u32)__popcll(nv & ~old);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  wave_count(pop, newbits);
  if (changed) {
    const u64 any = __ballot(ch);
    if (any && lane == 0) atomicOr(changed, 1u);
  }
}

}  // namespace

i64 gemm_mfma_max_kwords() { return kMaxKWords; }

hipError_t launch_gemm_mfma(const GemmArgs& g, const u64* BT, i64 ldbt, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (words_for(g.K) > kMaxKWords) return hipErrorInvalidValue;
  const i64 tiles = ((g.M + kMT - 1) / kMT) * ((g.N + kMT - 1) / kMT);
  hipLaunchKernelGGL(k_gemm_mfma, dim3((unsigned)tiles), dim3(512), 0, s, g.A, g.lda, BT, ldbt, g.Cold, g.ldco, g.C,
                     g.ldc, g.D, g.ldd, g.M, g.K, g.N, g.changed, g.newbits, g.pred, g.pred_val);
  return hipGetLastError();
}


hipError_t launch_gemm_valu(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  constexpr i64 kTargetBlocks = 1024;  // 4 workgroups per CU on 256 CUs
  if (g.M <= 64) return launch_rpw<4>(g, s, kTargetBlocks);
  return launch_rpw<16>(g, s, kTargetBlocks);
}

}  // namespace bmlp
