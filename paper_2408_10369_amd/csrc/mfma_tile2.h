// The matrix-core Boolean product tile, second layout: raw bit words staged in LDS, operands formed in
// registers.  Shared by the single-product kernel's tuned variants.  Not part of the public C-ABI.
#pragma once
#include "bmlp_internal.h"
#include "mfma_tile.h"

namespace bmlp {

// ---------------------------------------------------------------------------
// Same arithmetic as mfma_tile (v_mfma_scale_f32_32x32x64_f8f6f4, e2m1 operands, scales 2^0, "> 0" on
// the fp32 sums), different data movement:
//
//  * LDS holds the operands' bit words as loaded (no 4x expansion), so a chunk of KC words of k costs
//    256 rows x 8 KC bytes per operand.  Each row is stored half-planar: the low dwords of its KC words,
//    then the high dwords, in 16-byte units of four words.  Units are XOR-swizzled by the row so that
//    the 8 (or 16) rows that one LDS cycle serves fall on distinct banks (checked on the host for 32 and
//    64 banks of 4 bytes).
//  * Global loads are coalesced: KC / 2 lanes cover one row's KC words with 16-byte loads (whole 128- or
//    64-byte segments), and each wave stages 64 rows of A or of B^T per chunk.
//  * A consuming lane (row l32 of a 32 x 32 block, lane half h) reads the half-h dwords of four words
//    with one 16-byte LDS load and forms the e2m1 operand of each word in registers.  With the half-h
//    dword x of a word, the four operand dwords are
//        SUB = 1: x & 0x11111111 (0.5), x & 0x22222222 (1.0), x & 0x44444444 (2.0), (x >> 1) & 0x44444444
//        SUB = 0: x & 0x22222222, x & 0x44444444, (x >> 2) & 0x22222222, (x << 2) & 0x44444444
//    so every nibble carries exactly one bit of the word at a place worth a positive value (the sign
//    place 0b1000 is never used), each of the 32 bits once.  A and B^T share the map, so a product term
//    is positive exactly when both bits are set, and a sum of non-negative terms is positive exactly when
//    one of them is: the OR of ANDs, whatever the hardware's order of summation and its rounding.
//  * Zero words: while staging, each wave ballots which of the chunk's words are nonzero in its 64 rows;
//    a consuming wave skips a group of four words that are all zero in all 128 of its A rows or all 64
//    of its B^T rows.
//  * The kernel needs 16-byte aligned rows of A and B^T (even leading dimensions, aligned bases).
//  * Tiles whose C_old is all ones are copied; waves vote on saturation and the workgroup stops early
//    (as in mfma_tile); the epilogue is the same.  When A is known to be dense (MfmaTile::early),
//    a whole tile votes right after its first chunk, before loading the next.
template <int KC>
struct Mfma2Lds {
  static_assert(KC == 8 || KC == 16, "KC is 8 or 16 words");  // 16 needs more registers than two waves per SIMD have
  u32 X[2][2][kMT][2 * KC];  // stage, operand (0: A, 1: B^T), row, swizzled half-planar dwords
  u64 bal[8][2][16];
  u64 cold[kMT][4];  // the tile's C_old words, kept by tile_cold_full
  u32 zmask[2][8];  // per stage and staging wave: bit q = word q of the chunk is nonzero in the wave's rows
  u32 satf[2][8];
  u64 cnt[8][3];  // per wave: new bits, words of k multiplied, changed (tile_counters)
};

// physical 16-byte unit of logical unit u (u = half * KC / 8 + word / 4) in row r
template <int KC>
__device__ __forceinline__ int mfma2_unit(int u, int r) {
  if (KC == 16) return u ^ ((r ^ (r >> 3)) & 7);
  return u ^ (((r >> 1) ^ (r >> 3)) & 3);
}

__device__ __forceinline__ v8i_t mfma2_operand_sub(u32 x) {
  return v8i_t{(int)(x & 0x11111111u), (int)(x & 0x22222222u), (int)(x & 0x44444444u),
               (int)((x >> 1) & 0x44444444u), 0, 0, 0, 0};
}
__device__ __forceinline__ v8i_t mfma2_operand_nosub(u32 x) {
  return v8i_t{(int)(x & 0x22222222u), (int)(x & 0x44444444u), (int)((x >> 2) & 0x22222222u),
               (int)((x << 2) & 0x44444444u), 0, 0, 0, 0};
}
template <int SUB>
__device__ __forceinline__ v8i_t mfma2_operand(u32 x) {
  return SUB ? mfma2_operand_sub(x) : mfma2_operand_nosub(x);
}

// Output tile (tr, tc) of C = Cold | A.B (256 x 256) by one workgroup of 512 threads.  Every thread of
// the workgroup must call it with the same tile.
template <int KC, int SUB>
__device__ __forceinline__ void mfma_tile2(Mfma2Lds<KC>& L, const MfmaTile& g, i64 tr, i64 tc) {
  constexpr int U = KC / 2;        // 16-byte units per staged row
  constexpr int LPR = KC / 2;      // staging lanes per row (16 bytes = 2 words each)
  constexpr int RPI = 64 / LPR;    // rows per staging load instruction of a wave
  const u64* __restrict__ A = g.A;
  const u64* __restrict__ BT = g.BT;
  const u64* __restrict__ Cold = g.Cold;
  const i64 M = g.M, K = g.K, N = g.N;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;  // consumer: rows wr*128 .. +128, columns wc*64 .. +64
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

  // staging: waves 0..3 stage A rows 64 w .. +64, waves 4..7 B^T rows 64 (w - 4) .. +64 of the tile, NL
  // loads of 16 bytes (words 2p and 2p + 1 of a row) per thread and chunk, RPI rows per load instruction
  constexpr int NL = 64 / RPI;
  const bool isa = wave < 4;
  const int srow_base = (wave & 3) * 64;
  const int p = lane % LPR;
  const int rsub = lane / LPR;
  const i64 ldsrc = isa ? g.lda : g.ldbt;
  const i64 rlim = isa ? M : N;
  const i64 r0 = (isa ? row0 : col0) + srow_base + rsub;  // this lane's first staged row
  const u64* __restrict__ src = (isa ? A : BT) + (r0 < rlim ? r0 : 0) * ldsrc;
  const i64 nchunks = (kwords + KC - 1) / KC;
  uint4 sr[NL];
  auto load = [&](i64 chunk) {
    const i64 w = chunk * KC + 2 * p;  // first word of this lane's piece
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const bool v = r0 + j * RPI < rlim;
      const u64* pr = src + (v ? (i64)(j * RPI) * ldsrc : 0);
      if (v && w + 1 < kwords) {
        sr[j] = *(const uint4*)(pr + w);
      } else if (v && w < kwords) {
        const u64 x = pr[w];
        sr[j] = make_uint4((u32)x, (u32)(x >> 32), 0u, 0u);
      } else {
        sr[j] = make_uint4(0u, 0u, 0u, 0u);
      }
    }
  };
  // write the loaded chunk into stage buf (half-planar, swizzled) and record its nonzero words
  auto stage = [&](int buf) {
    u32(*X)[2 * KC] = L.X[buf][isa ? 0 : 1];
    const int u = p >> 1, off = 2 * (p & 1);  // logical unit of words 2p, 2p + 1, dword offset in it
    u32 mine = 0;  // bit 0: word 2p nonzero in one of this lane's rows; bit 1: word 2p + 1
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int r = srow_base + j * RPI + rsub;
      *(uint2*)&X[r][4 * mfma2_unit<KC>(u, r) + off] = make_uint2(sr[j].x, sr[j].z);          // low dwords
      *(uint2*)&X[r][4 * mfma2_unit<KC>(U / 2 + u, r) + off] = make_uint2(sr[j].y, sr[j].w);  // high dwords
      mine |= ((sr[j].x | sr[j].y) != 0u ? 1u : 0u) | ((sr[j].z | sr[j].w) != 0u ? 2u : 0u);
    }
    // bit q of the mask: word q of the chunk is nonzero in some row this wave staged (lanes l with
    // l % LPR == q' hold words 2q' and 2q' + 1)
    const u64 b0 = __ballot(mine & 1u), b1 = __ballot(mine & 2u);
    u32 zm = 0;
#pragma unroll
    for (int q = 0; q < LPR; ++q) {
      u64 sel = 0;
#pragma unroll
      for (int rr = 0; rr < RPI; ++rr) sel |= 1ull << (rr * LPR + q);
      if (b0 & sel) zm |= 1u << (2 * q);
      if (b1 & sel) zm |= 1u << (2 * q + 1);
    }
    if (lane == 0) L.zmask[buf][wave] = zm;
  };
  u32 done_words = 0;  // words of k this wave ran the matrix cores on
  // consume stage buf: four words per 16-byte read of every block's row.  Groups of four words are skipped
  // when all four are zero on one side; inside a group every word is multiplied (a zero word adds
  // nothing).  The reads of group gq + 1 are issued before the products of group gq, and every operand
  // of a word is formed before its eight products, so that the products go back to back.
  auto read_group = [&](int buf, int gq, uint4 (&av)[4], uint4 (&bv)[2]) {
    const u32(*XA)[2 * KC] = L.X[buf][0];
    const u32(*XB)[2 * KC] = L.X[buf][1];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wr * 128 + i * 32 + l32;
      av[i] = *(const uint4*)&XA[r][4 * mfma2_unit<KC>(h * (U / 2) + gq, r)];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int r = wc * 64 + j * 32 + l32;
      bv[j] = *(const uint4*)&XB[r][4 * mfma2_unit<KC>(h * (U / 2) + gq, r)];
    }
  };
  auto compute = [&](int buf, u32 mask) {
    uint4 av[4], bv[2];
    read_group(buf, 0, av, bv);
#pragma unroll
    for (int gq = 0; gq < KC / 4; ++gq) {
      uint4 an[4], bn[2];
      if (gq + 1 < KC / 4) read_group(buf, gq + 1, an, bn);
      if (((mask >> (4 * gq)) & 15u) != 0u) {
        done_words += 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v8i_t bf[2], af[4];
#pragma unroll
          for (int j = 0; j < 2; ++j)
            bf[j] = mfma2_operand<SUB>(e == 0 ? bv[j].x : e == 1 ? bv[j].y : e == 2 ? bv[j].z : bv[j].w);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            af[i] = mfma2_operand<SUB>(e == 0 ? av[i].x : e == 1 ? av[i].y : e == 2 ? av[i].z : av[i].w);
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[i], bf[j], acc[i][j], 4, 4, 0, 127, 0, 127);
        }
      }
      if (gq + 1 < KC / 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = an[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = bn[j];
      }
    }
  };
  const bool whole = row0 + kMT <= M && col0 + kMT <= N;
  bool wsat = false;  // wave-uniform
  // words of chunk buf to multiply (wave-uniform): none once the wave is saturated
  auto chunk_mask = [&](int buf) -> u32 {
    return wsat ? 0u
                : __builtin_amdgcn_readfirstlane((L.zmask[buf][2 * wr] | L.zmask[buf][2 * wr + 1]) &
                                                 L.zmask[buf][4 + wc]);
  };
  // the wave is saturated once every one of its sums is positive
  auto update_wsat = [&]() {
    if (wsat) return;
    float mn = acc[0][0][0];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) mn = fminf(mn, acc[i][j][e]);
    wsat = __ballot(!(mn > 0.f)) == 0ull;
  };
  load(0);
  // the first loads are in flight while the C_old check waits for its words
  if (Cold && tile_cold_full(L.cold, g, row0, col0)) return;
  stage(0);
  int pending = -1;
  int votes = 0;
  i64 c0 = 0;
  if (whole && nchunks > 1 && (g.early || (g.early_flag && *g.early_flag != 0u))) {
    // A is dense: the first chunk alone likely saturates the tile, so it is consumed and voted on
    // before any further chunk is loaded (a chunk loaded ahead would hold the workgroup until it arrived).
    // A tile that is not saturated then starts the pipeline at chunk 1.
    __syncthreads();
    compute(0, chunk_mask(0));
    update_wsat();
    if (lane == 0) L.satf[0][wave] = wsat ? 1u : 0u;
    __syncthreads();
    u32 all = 1u;
#pragma unroll
    for (int w = 0; w < 8; ++w) all &= L.satf[0][w];
    if (all) {
      c0 = nchunks;
    } else {
      load(1);
      stage(1);
      if (2 < nchunks) load(2);
      c0 = 1;
      votes = 1;
    }
  } else if (1 < nchunks) {
    load(1);
  }
  for (i64 c = c0; c < nchunks; ++c) {
    __syncthreads();
    if (pending >= 0) {
      u32 all = 1u;
#pragma unroll
      for (int w = 0; w < 8; ++w) all &= L.satf[pending][w];
      if (all) break;
      pending = -1;
    }
    const int buf = (int)(c & 1);
    if (c + 1 < nchunks) {
      stage(buf ^ 1);
      if (c + 2 < nchunks) load(c + 2);
    }
    compute(buf, chunk_mask(buf));
    // votes after 1, 2, 4, 8, ... chunks
    if (whole && ((c + 1) & c) == 0) {
      update_wsat();
      pending = votes & 1;
      if (lane == 0) L.satf[pending][wave] = wsat ? 1u : 0u;
      ++votes;
    }
  }

  tile_epilogue(acc, L.bal, Cold ? L.cold : nullptr, g, row0, col0, done_words, L.cnt);
}

}  // namespace bmlp
