// The matrix-core Boolean product tile shared by the single-product kernel and the batched rounds.
// Not part of the public C-ABI.
#pragma once
#include "bmlp_internal.h"
#include "valu_tile.h"

namespace bmlp {

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

// LDS of one tile (128 KiB + the C_old tile and the epilogue's ballots), declared once per kernel that uses mfma_tile
struct MfmaLds {
  uint4 Ax[2][2][kMT][kMChunk];  // per stage, lane half h, row and word slot: the dwords half h feeds in
  uint4 Bx[2][2][kMT][kMChunk];
  u64 bal[8][2][16];  // per wave: the ballots of a block row (tile_epilogue)
  u64 cold[kMT][4];  // the tile's C_old words (row, word of the tile), kept by tile_cold_full
  u32 zmask[2][8];  // per stage and staging wave (A: 0..3, B^T: 4..7): bit q = some row has a nonzero word q
  u32 satf[2][8];   // per vote (alternating) and wave: every output of the wave's 128 x 64 block is set
  u64 cnt[8][3];    // per wave: new bits, words of k multiplied, changed (tile_counters)
};

struct MfmaTile {
  const u64* A; i64 lda;
  const u64* BT; i64 ldbt;
  const u64* Cold; i64 ldco;
  u64* C; i64 ldc;
  u64* D; i64 ldd;
  i64 M, K, N;
  u32* changed;
  unsigned long long* newbits;
  unsigned long long* executed;
  u32* changed2;  // optional second flag set with *changed
  // the second tile code: a whole tile votes after its first chunk, before loading ahead, when early is
  // nonzero or *early_flag is (A is dense, so the tiles likely saturate there)
  const u32* early_flag = nullptr;
  u32 early = 0;
};

// Adds a tile's counts to the launch's counters (new bits, matrix-core work issued, the changed flags) with
// one device atomic per counter and workgroup: the eight waves' sums meet in LDS first.  Same-address device
// atomics are serialised; one per wave and counter (32,768 waves for a 16,384-node squaring) cost about a
// quarter of a millisecond on a launch whose tiles saturate early and otherwise take 0.2 ms.  Every thread of
// the workgroup calls it; pop is the lane's count, words and ch are wave-uniform.  The slots are read back
// before any thread can reach the next tile's epilogue (the K loop has a barrier).
__device__ __forceinline__ void tile_counters(u64 (&cnt)[8][3], const MfmaTile& g, u32 pop, u32 words, int ch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  u64 s = pop;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const u64 any = __ballot(ch);
  if (lane == 0) {
    cnt[wave][0] = s;
    cnt[wave][1] = words;
    cnt[wave][2] = any != 0ull ? 1ull : 0ull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 p = 0, w = 0, c = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      p += cnt[i][0];
      w += cnt[i][1];
      c |= cnt[i][2];
    }
    if (g.newbits && p) atomicAdd(g.newbits, (unsigned long long)p);
    // matrix-core work actually issued: 8 blocks of 32 x 32 x 64 MACs (2 ops each) per word and wave
    if (g.executed && w) atomicAdd(g.executed, (unsigned long long)w * 8ull * 131072ull);
    if (g.changed && c) {
      atomicOr(g.changed, 1u);
      if (g.changed2) atomicOr(g.changed2, 1u);
    }
  }
}

// Reads the C_old words of output tile (row0, col0), 256 rows of 4 words: thread t takes words t and
// t + 512 (row e / 4, word e % 4) and keeps them in `cold` for the epilogue.  Returns, the same in every
// thread, whether every bit of the tile is set; such a tile is final (C = C_old whatever A.B adds), and it
// is copied to C (and D cleared) here.  Every thread of the 512 must call it; it ends with a barrier.
__device__ __forceinline__ bool tile_cold_full(u64 (&cold)[kMT][4], const MfmaTile& g, i64 row0, i64 col0) {
  static_assert(kMT * 4 == 2 * 512, "two C_old words per thread");
  const int t = threadIdx.x;
  const i64 nw = (g.N + 63) >> 6;
  const u64 last_mask = (g.N & 63) ? ((1ull << (g.N & 63)) - 1ull) : ~0ull;
  u64 v[2];
  bool in[2];
  int full = 1;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = t + 512 * k;
    const i64 row = row0 + (e >> 2), w = (col0 >> 6) + (e & 3);
    in[k] = row < g.M && w < nw;
    v[k] = in[k] ? g.Cold[row * g.ldco + w] : 0ull;
    if (in[k]) full &= v[k] == (w == nw - 1 ? last_mask : ~0ull);
    cold[e >> 2][e & 3] = v[k];
  }
  if (!__syncthreads_and(full)) return false;
  const bool copy = g.C != g.Cold || g.ldc != g.ldco;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = t + 512 * k;
    const i64 row = row0 + (e >> 2), w = (col0 >> 6) + (e & 3);
    if (in[k]) {
      if (copy) g.C[row * g.ldc + w] = v[k];
      if (g.D) g.D[row * g.ldd + w] = 0ull;
    }
  }
  return true;
}

// s_waitcnt lgkmcnt(0), with vmcnt and expcnt at their maxima (gfx9 encoding): waits for LDS, not for memory
constexpr int kWaitLdsOnly = 0xC07F;

// The tile's epilogue: C = C_old | (sum > 0), D = C & ~C_old, then the counters.  A 32 x 32 fp32 block sits
// in lane l as column l % 32, register r holding row 8 (r / 4) + 4 (l / 32) + r % 4, so a ballot of "> 0" on
// register r holds columns 0..31 of two rows: 8 (r / 4) + r % 4 in its low half and the row 4 below in its
// high half.  Lane 0 keeps the ballots of a block row in LDS (bal, per wave); lane rho < 32 then assembles
// row rho's word of C from the two blocks side by side (columns 0..31 and 32..63).  Only LDS is waited
// for: the stores of C are never waited on, and C_old comes from LDS (tile_cold_full's copy).  cold: that
// copy, or null for C_old = 0.  Every thread of the 512 must call it.
__device__ __forceinline__ void tile_epilogue(const v16f_t (&acc)[4][2], u64 (&bal)[8][2][16], const u64 (*cold)[4],
                                              const MfmaTile& g, i64 row0, i64 col0, u32 done_words,
                                              u64 (&cnt)[8][3]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int rho = lane & 31;
  const int hh = (rho >> 2) & 1, r = ((rho >> 3) << 2) | (rho & 3);  // rho = 8 (r / 4) + 4 hh + r % 4
  const i64 nw = (g.N + 63) >> 6;
  const i64 w = (col0 >> 6) + wc;
  int ch = 0;
  u32 pop = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const u64 b = __ballot(acc[i][j][q] > 0.f);
        if (lane == 0) bal[wave][j][q] = b;
      }
    }
    // the lanes below read what lane 0 of the same wave wrote (LDS keeps a wave's order)
    __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);
    __builtin_amdgcn_wave_barrier();
    const int trow = wr * 128 + i * 32 + rho;
    const i64 row = row0 + trow;
    if (lane < 32 && row < g.M && w < nw) {
      const u64 word = ((bal[wave][0][r] >> (32 * hh)) & 0xFFFFFFFFull) |
                       (((bal[wave][1][r] >> (32 * hh)) & 0xFFFFFFFFull) << 32);
      const u64 old = cold ? cold[trow][wc] : 0ull;
      const u64 nv = word | old;
      g.C[row * g.ldc + w] = nv;
      if (g.D) g.D[row * g.ldd + w] = nv & ~old;
      ch |= (nv != old);
      pop += (u32)__popcll(nv & ~old);
    }
    __builtin_amdgcn_wave_barrier();
  }
  tile_counters(cnt, g, pop, done_words, ch);
}

// Output tile (tr, tc) of C = Cold | A.B (256 x 256) by one workgroup of 512 threads.  Every thread of
// the workgroup must call it with the same tile.
__device__ __forceinline__ void mfma_tile(MfmaLds& L, const MfmaTile& g, i64 tr, i64 tc) {
  const u64* __restrict__ A = g.A;
  const i64 lda = g.lda;
  const u64* __restrict__ BT = g.BT;
  const i64 ldbt = g.ldbt;
  const u64* __restrict__ Cold = g.Cold;
  const i64 M = g.M, K = g.K, N = g.N;
  auto& Ax = L.Ax;
  auto& Bx = L.Bx;
  auto& zmask = L.zmask;
  auto& satf = L.satf;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;  // wave owns rows wr*128 .. +128, columns wc*64 .. +64
  const int h = lane >> 5, l32 = lane & 31;
  const i64 row0 = tr * kMT, col0 = tc * kMT;
  const i64 kwords = (K + 63) >> 6;

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
  auto stage_word = [&](const u64 (&sr)[kMChunk], int buf, int q) -> u32 {
    uint4 (*X)[kMT][kMChunk] = isa ? Ax[buf] : Bx[buf];
    const u32 lo = (u32)sr[q], hi = (u32)(sr[q] >> 32), rlo = rotr2(lo), rhi = rotr2(hi);
    const int slot = q ^ ssw;
    X[0][tt][slot] = make_uint4(lo & 0x22222222u, hi & 0x22222222u, lo & 0x44444444u, hi & 0x44444444u);
    X[1][tt][slot] = make_uint4(rlo & 0x22222222u, rhi & 0x22222222u, rlo & 0x44444444u, rhi & 0x44444444u);
    return __ballot(sr[q] != 0ull) != 0ull ? (1u << q) : 0u;
  };
  auto stage = [&](const u64 (&sr)[kMChunk], int buf) {
    u32 zm = 0;
#pragma unroll
    for (int q = 0; q < kMChunk; ++q) zm |= stage_word(sr, buf, q);
    if (lane == 0) zmask[buf][wave] = zm;
  };
  u32 done_words = 0;  // words of k this wave ran the matrix cores on
  const int csw = (l32 >> 2) & 3;  // word-slot swizzle of every row this lane reads
  // the staging of the next chunk (sn into stage buf ^ 1) is interleaved word by word with the MFMA groups
  auto compute = [&](int buf, uint4 (&av)[4], uint4 (&bv)[2], u32 mask, const u64 (&sn)[kMChunk], bool next) {
    const uint4* as = &Ax[buf][h][wr * 128 + l32][0];
    const uint4* bs = &Bx[buf][h][wc * 64 + l32][0];
    done_words += __builtin_popcount(mask);
    u32 zm = 0;
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
      if (next) zm |= stage_word(sn, buf ^ 1, q);
      if (q + 1 < kMChunk) {
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = an[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = bn[j];
      }
    }
    if (next && lane == 0) zmask[buf ^ 1][wave] = zm;
  };
  // Saturation: the sums only grow, so once every accumulator of a wave is positive its 128 x 64 outputs
  // are final (all ones), and the wave stops issuing matrix-core work.  The waves vote now and then (see
  // the loop); a vote is read after the next barrier, and once all eight waves are saturated the
  // workgroup leaves the loop (only whole tiles vote: rows or columns past the matrix never fill).
  const bool whole = row0 + kMT <= M && col0 + kMT <= N;
  bool wsat = false;  // wave-uniform
  // sn holds chunk c + 1 on entry; on exit it holds (the loads of) chunk c + 3.  Returns whether every
  // wave of the workgroup reported saturation in the last vote (the same answer in every thread).
  auto step = [&](u64 (&sn)[kMChunk], i64 c, int vote) -> bool {
    __syncthreads();
    if (vote >= 0) {
      u32 all = 1u;
#pragma unroll
      for (int w = 0; w < 8; ++w) all &= satf[vote][w];
      if (all) return true;
    }
    const int buf = (int)(c & 1);
    // the first word's operands and the skip mask of chunk c are read before the staging of chunk c + 1,
    // so that their LDS latency overlaps it
    uint4 av[4], bv[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = Ax[buf][h][wr * 128 + l32 + 32 * i][0 ^ csw];
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = Bx[buf][h][wc * 64 + l32 + 32 * j][0 ^ csw];
    // words q of k with a nonzero word in some row of this wave's A rows and in some of its B^T rows
    // (wave-uniform): a word that is zero on either side adds nothing to any of the wave's sums
    const u32 mask = wsat ? 0u
                          : __builtin_amdgcn_readfirstlane((zmask[buf][2 * wr] | zmask[buf][2 * wr + 1]) &
                                                           zmask[buf][4 + wc]);
    const bool next = c + 1 < nchunks;
    compute(buf, av, bv, mask, sn, next);
    if (next && c + 3 < nchunks) load(sn, c + 3);
    return false;
  };
  load(s0, 0);
  load(s1, 1);
  // the first loads are in flight while the C_old check waits for its words
  if (Cold && tile_cold_full(L.cold, g, row0, col0)) return;
  stage(s0, 0);
  if (2 < nchunks) load(s0, 2);
  int pending = -1;  // vote slot to read after the next barrier
  int votes = 0;
  for (i64 c = 0, it = 0; c < nchunks; c += 2, ++it) {
    if (step(s1, c, pending)) break;
    pending = -1;
    if (c + 1 < nchunks) step(s0, c + 1, -1);
    // votes after 2, 4, 8, 16, ... chunks: a product that saturates does so early, and one that does not
    // pays for a handful of checks only
    if (whole && ((it + 1) & it) == 0) {
      if (!wsat) {
        float mn = acc[0][0][0];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) mn = fminf(mn, acc[i][j][e]);
        wsat = __ballot(!(mn > 0.f)) == 0ull;
      }
      pending = votes & 1;
      if (lane == 0) satf[pending][wave] = wsat ? 1u : 0u;
      ++votes;
    }
  }

  tile_epilogue(acc, L.bal, Cold ? L.cold : nullptr, g, row0, col0, done_words, L.cnt);
}

}  // namespace bmlp
