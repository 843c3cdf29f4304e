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
// MFMA arm: 4-bit (e2m1) matrix cores, fp32 accumulation, "> 0" threshold.
//
// The operands stay bit-packed in memory.  One v_mfma_scale_f32_32x32x64_f8f6f4
// with both operands in the e2m1 format (scales 2^0) takes 64 k-values for each
// of 32 rows, 32 per lane: lane half h = lane / 32 feeds 4 dwords of 8 nibbles.
// A nibble that carries one bit of the relation in place holds 0 or one of
// 0b0010 (1.0) and 0b0100 (2.0); the other two places would be the sign (0b1000)
// and a subnormal (0b0001), so they are moved: each 32-bit half w of a word is
// also used rotated right by 2, and
//     h = 0: { lo & 0x22222222, hi & 0x22222222, lo & 0x44444444, hi & 0x44444444 }
//     h = 1: the same masks applied to rotr(lo, 2), rotr(hi, 2)
// (bits 4n+1, 4n+2 as loaded; bits 4n+3, 4n+4 after the rotation), so the two
// halves of the wave cover all 64 bits of one word of k.  A and B^T use the
// same bit -> (lane half, nibble, value) map, so every product term is 0,
// 1 * 1 or 2 * 2, all exact, and the fp32 sum -- an integer at most 4 K, exact
// while 4 K <= 2^24, i.e. for up to kMaxKWords words of k -- is positive exactly
// when some k has A_ik = B_kj = 1: the OR of ANDs.  A sum does not depend on
// the order of its terms, so the result is exact whatever k order the
// instruction assigns to (half, nibble); it only has to be the same for both
// operands.  B is consumed transposed (B^T rows = columns of B), so that a
// column's 64 k-bits are one word, like a row of A.  (The 32 x 32 x 64 shape
// runs the 4-bit format at twice the 8-bit rate; the 16 x 16 x 128 shape does
// not.)
//
// Tile: a workgroup of 8 waves (two per SIMD) owns 256 x 256 outputs; wave
// (wr, wc) owns rows 128 wr .. +128 and columns 64 wc .. +64 = 4 x 2 MFMA
// blocks of 32 x 32.  Per chunk of kMChunk words of k the workgroup stages 256
// rows of A (threads 0..255) and 256 rows of B^T (threads 256..511) in LDS as
// ready operands: for every row, word and lane half the 4 masked dwords above,
// so a consuming lane reads its operand with one 16-byte LDS load and spends no
// ALU on it.  LDS stages are double-buffered and software-pipelined: after the
// barrier that opens chunk c the threads stage chunk c + 1 into the other buffer
// (its global loads were issued two chunks earlier) while the waves consume
// chunk c, so one barrier per chunk suffices.  Word slots are XOR-swizzled
// by bits 2-3 of the row so that the 16 rows a quarter-wave reads fall on
// distinct LDS banks.  While staging, the A waves also record which words of
// the chunk are nonzero in any of their rows; a consuming wave skips the words
// where all 128 of its rows are zero.
typedef float v16f_t __attribute__((ext_vector_type(16)));
typedef int v8i_t __attribute__((ext_vector_type(8)));

constexpr int kMT = 256;     // workgroup tile (rows and columns)
constexpr int kMChunk = 4;   // words of k per LDS stage (one word per 32 x 32 x 64 MFMA step)
constexpr i64 kMaxKWords = 65536;  // sums <= 4 K <= 2^24 stay exact in fp32

__device__ __forceinline__ u32 rotr2(u32 x) { return __builtin_amdgcn_alignbit(x, x, 2); }

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_mfma(const u64* __restrict__ A, i64 lda, const u64* __restrict__ BT, i64 ldbt, const u64* __restrict__ Cold,
            i64 ldco, u64* __restrict__ C, i64 ldc, u64* __restrict__ D, i64 ldd, i64 M, i64 K, i64 N,
            u32* __restrict__ changed, unsigned long long* __restrict__ newbits, const u32* __restrict__ pred,
            u32 pred_val, unsigned long long* __restrict__ executed) {
  // per stage, lane half h, row and word slot: the 4 dwords lane half h feeds to the MFMA
  __shared__ uint4 Ax[2][2][kMT][kMChunk];
  __shared__ uint4 Bx[2][2][kMT][kMChunk];
  __shared__ u64 bal[8][2][16];
  __shared__ u32 zmask[2][4];  // per stage and A-staging wave: bit q = some row has a nonzero word q
  if (pred && *pred != pred_val) return;  // another arm serves this round
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;  // wave owns rows wr*128 .. +128, columns wc*64 .. +64
  const int h = lane >> 5, l32 = lane & 31;
  const i64 ctiles = (N + kMT - 1) / kMT;
  const i64 tr = blockIdx.x / ctiles, tc = blockIdx.x % ctiles;
  const i64 row0 = tr * kMT, col0 = tc * kMT;
  const i64 kwords = (K + 63) >> 6;
  const i64 nw = (N + 63) >> 6;

  // A tile whose C_old bits are all set is final (C = C_old whatever A.B adds): copy it and stop.
  if (Cold) {
    const u64 last_mask = (N & 63) ? ((1ull << (N & 63)) - 1ull) : ~0ull;
    int full = 1;
    for (int e = t; e < kMT * 4; e += 512) {
      const i64 row = row0 + (e >> 2), w = (col0 >> 6) + (e & 3);
      if (row < M && w < nw) full &= Cold[row * ldco + w] == (w == nw - 1 ? last_mask : ~0ull);
    }
    if (__syncthreads_and(full)) {
      const bool copy = C != Cold || ldc != ldco;
      for (int e = t; e < kMT * 4; e += 512) {
        const i64 row = row0 + (e >> 2), w = (col0 >> 6) + (e & 3);
        if (row < M && w < nw) {
          if (copy) C[row * ldc + w] = Cold[row * ldco + w];
          if (D) D[row * ldd + w] = 0ull;
        }
      }
      return;
    }
  }

  v16f_t acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // threads 0..255 stage row t of the A tile, threads 256..511 row t-256 of the B^T tile
  const bool isa = t < 256;
  const int tt = t & 255;
  const i64 rr = (isa ? row0 : col0) + tt;
  const bool vr = rr < (isa ? M : N);
  const u64* pr = isa ? A + (vr ? rr : 0) * lda : BT + (vr ? rr : 0) * ldbt;
  const int ssw = (tt >> 2) & 3;  // word-slot swizzle of the staged row
  // Software pipeline over chunks of kMChunk words: after the barrier that opens chunk c, every thread
  // stages chunk c + 1 (already in registers) into the other LDS buffer and issues the global loads of
  // chunk c + 3, then the waves consume chunk c.  Two register sets alternate, so a load has two chunk
  // times to arrive before it is staged.
  const i64 nchunks = (kwords + kMChunk - 1) / kMChunk;
  u64 s0[kMChunk], s1[kMChunk];
  auto load = [&](u64 (&sr)[kMChunk], i64 chunk) {
    const i64 kb = chunk * kMChunk;
#pragma unroll
    for (int q = 0; q < kMChunk; ++q) sr[q] = (vr && kb + q < kwords) ? pr[kb + q] : 0ull;
  };
  auto stage = [&](const u64 (&sr)[kMChunk], int buf) {
    uint4 (*X)[kMT][kMChunk] = isa ? Ax[buf] : Bx[buf];
#pragma unroll
    for (int q = 0; q < kMChunk; ++q) {
      const u32 lo = (u32)sr[q], hi = (u32)(sr[q] >> 32), rlo = rotr2(lo), rhi = rotr2(hi);
      const int slot = q ^ ssw;
      X[0][tt][slot] = make_uint4(lo & 0x22222222u, hi & 0x22222222u, lo & 0x44444444u, hi & 0x44444444u);
      X[1][tt][slot] = make_uint4(rlo & 0x22222222u, rhi & 0x22222222u, rlo & 0x44444444u, rhi & 0x44444444u);
    }
    if (isa) {
      u32 zm = 0;
#pragma unroll
      for (int q = 0; q < kMChunk; ++q) zm |= (__ballot(sr[q] != 0ull) != 0ull ? 1u : 0u) << q;
      if (lane == 0) zmask[buf][wave] = zm;
    }
  };
  u32 done_words = 0;  // words of k this wave ran the matrix cores on
  const int csw = (l32 >> 2) & 3;  // word-slot swizzle of every row this lane reads
  auto compute = [&](int buf, uint4 (&av)[4], uint4 (&bv)[2], u32 mask) {
    const uint4* as = &Ax[buf][h][wr * 128 + l32][0];
    const uint4* bs = &Bx[buf][h][wc * 64 + l32][0];
    done_words += __builtin_popcount(mask);
    // operands of word q + 1 are read while word q is consumed
#pragma unroll
    for (int q = 0; q < kMChunk; ++q) {
      uint4 an[4], bn[2];
      if (q + 1 < kMChunk) {
#pragma unroll
        for (int i = 0; i < 4; ++i) an[i] = as[i * 32 * kMChunk + ((q + 1) ^ csw)];
#pragma unroll
        for (int j = 0; j < 2; ++j) bn[j] = bs[j * 32 * kMChunk + ((q + 1) ^ csw)];
      }
      if ((mask >> q) & 1u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const v8i_t af = v8i_t{(int)av[i].x, (int)av[i].y, (int)av[i].z, (int)av[i].w, 0, 0, 0, 0};
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const v8i_t bf = v8i_t{(int)bv[j].x, (int)bv[j].y, (int)bv[j].z, (int)bv[j].w, 0, 0, 0, 0};
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af, bf, acc[i][j], 4, 4, 0, 127, 0, 127);
          }
        }
      }
      if (q + 1 < kMChunk) {
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = an[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = bn[j];
      }
    }
  };
  // sn holds chunk c + 1 on entry; on exit it holds (the loads of) chunk c + 3
  auto step = [&](u64 (&sn)[kMChunk], i64 c) {
    __syncthreads();
    const int buf = (int)(c & 1);
    // the first word's operands and the skip mask of chunk c are read before the staging of chunk c + 1,
    // so that their LDS latency overlaps it
    uint4 av[4], bv[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = Ax[buf][h][wr * 128 + l32 + 32 * i][0 ^ csw];
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = Bx[buf][h][wc * 64 + l32 + 32 * j][0 ^ csw];
    // rows of this wave with a nonzero word q of k (wave-uniform)
    const u32 mask = __builtin_amdgcn_readfirstlane(zmask[buf][2 * wr] | zmask[buf][2 * wr + 1]);
    if (c + 1 < nchunks) {
      stage(sn, buf ^ 1);
      if (c + 3 < nchunks) load(sn, c + 3);
    }
    compute(buf, av, bv, mask);
  };
  load(s0, 0);
  load(s1, 1);
  stage(s0, 0);
  if (2 < nchunks) load(s0, 2);
  for (i64 c = 0; c < nchunks; c += 2) {
    step(s1, c);
    if (c + 1 < nchunks) step(s0, c + 1);
  }

  // epilogue: a 32 x 32 fp32 block sits in lane l as column l % 32, register r holding row
  // 8 (r / 4) + 4 (l / 32) + r % 4; ballot "> 0" per register, assemble 32 rows x 1 word per block row
  int ch = 0;
  u32 pop = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const u64 b = __ballot(acc[i][j][r] > 0.f);
        if (lane == 0) bal[wave][j][r] = b;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (lane < 32) {
      const int rho = lane;  // row within the block: rho = 8 (r / 4) + 4 hh + r % 4
      const int hh = (rho >> 2) & 1, r = ((rho >> 3) << 2) | (rho & 3);
      const u64 word = ((bal[wave][0][r] >> (32 * hh)) & 0xFFFFFFFFull) |
                       (((bal[wave][1][r] >> (32 * hh)) & 0xFFFFFFFFull) << 32);
      const i64 row = row0 + wr * 128 + i * 32 + rho;
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
  // matrix-core work actually issued: 8 blocks of 32 x 32 x 64 MACs (2 ops each) per word
  if (executed && lane == 0 && done_words) atomicAdd(executed, (unsigned long long)done_words * 8ull * 131072ull);
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
                     g.ldc, g.D, g.ldd, g.M, g.K, g.N, g.changed, g.newbits, g.pred, g.pred_val, g.executed);
  return hipGetLastError();
}


hipError_t launch_gemm_valu(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  constexpr i64 kTargetBlocks = 1024;  // 4 workgroups per CU on 256 CUs
  if (g.M <= 64) return launch_rpw<4>(g, s, kTargetBlocks);
  return launch_rpw<16>(g, s, kTargetBlocks);
}

}  // namespace bmlp
