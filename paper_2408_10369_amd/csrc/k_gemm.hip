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
#include "bmlp_internal.h"

namespace bmlp {

namespace {

// all-ones when bit `b` of the wave-uniform word x is set, else zero
__device__ __forceinline__ u32 bit_mask(u32 x, int b) { return (u32)(((int)(x << (31 - b))) >> 31); }

// acc | (b & m) as one v_and_or_b32 (m is a scalar operand)
__device__ __forceinline__ u32 and_or(u32 b, u32 m, u32 acc) {
  u32 r;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(b), "s"(m), "v"(acc));
  return r;
}

template <int RPW, int WPL>
__global__ void __launch_bounds__(256)
k_gemm_valu(const u64* __restrict__ A, i64 lda, const u64* __restrict__ B, i64 ldb, const u64* __restrict__ Cold,
            i64 ldco, u64* __restrict__ C, i64 ldc, u64* __restrict__ D, i64 ldd, i64 M, i64 K, i64 N,
            u32* __restrict__ changed) {
  constexpr int TW = 64 * WPL;
  constexpr int TR = 4 * RPW;
  __shared__ u64 Bs[64][TW];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const i64 nw = (N + 63) >> 6;
  const i64 ctiles = (nw + TW - 1) / TW;
  const i64 tile = blockIdx.x;
  const i64 ct = tile % ctiles, rt = tile / ctiles;
  const i64 row0 = rt * TR + (i64)wave * RPW;
  const i64 w0 = ct * TW;

  u32 acc[RPW][WPL][2];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int wl = 0; wl < WPL; ++wl) acc[r][wl][0] = acc[r][wl][1] = 0u;

  const i64 kwords = (K + 63) >> 6;
  for (i64 kw = 0; kw < kwords; ++kw) {
    u32 alo[RPW], ahi[RPW];
    u32 any = 0;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const i64 row = row0 + r;
      const u64 a = (row < M) ? A[row * lda + kw] : 0ull;
      alo[r] = (u32)a;
      ahi[r] = (u32)(a >> 32);
      any |= alo[r] | ahi[r];
    }
    if (!__syncthreads_or(any != 0)) continue;
    for (int idx = threadIdx.x; idx < 64 * TW; idx += 256) {
      const int t = idx / TW, c = idx - (idx / TW) * TW;
      const i64 k = kw * 64 + t, w = w0 + c;
      Bs[t][c] = (k < K && w < nw) ? B[k * ldb + w] : 0ull;
    }
    __syncthreads();
    if (any) {
#pragma unroll
      for (int kk = 0; kk < 64; ++kk) {
        u32 blo[WPL], bhi[WPL];
#pragma unroll
        for (int wl = 0; wl < WPL; ++wl) {
          const u64 b = Bs[kk][lane + 64 * wl];
          blo[wl] = (u32)b;
          bhi[wl] = (u32)(b >> 32);
        }
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const u32 m = bit_mask(kk < 32 ? alo[r] : ahi[r], kk & 31);
#pragma unroll
          for (int wl = 0; wl < WPL; ++wl) {
            acc[r][wl][0] = and_or(blo[wl], m, acc[r][wl][0]);
            acc[r][wl][1] = and_or(bhi[wl], m, acc[r][wl][1]);
          }
        }
      }
    }
  }

  int ch = 0;
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const i64 row = row0 + r;
    if (row >= M) break;
#pragma unroll
    for (int wl = 0; wl < WPL; ++wl) {
      const i64 w = w0 + lane + 64 * wl;
      if (w < nw) {
        const u64 old = Cold ? Cold[row * ldco + w] : 0ull;
        const u64 v = (((u64)acc[r][wl][1] << 32) | (u64)acc[r][wl][0]) | old;
        C[row * ldc + w] = v;
        if (D) D[row * ldd + w] = v & ~old;
        ch |= (v != old);
      }
    }
  }
  if (changed) {
    const u64 bal = __ballot(ch);
    if (bal && lane == 0) atomicOr(changed, 1u);
  }
}

}  // namespace

hipError_t launch_gemm_valu(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const i64 nw = words_for(g.N);
  constexpr int RPW = 16;
  if (nw >= 64) {
    constexpr int WPL = 1;
    const i64 ctiles = (nw + 64 * WPL - 1) / (64 * WPL);
    const i64 rtiles = (g.M + 4 * RPW - 1) / (4 * RPW);
    hipLaunchKernelGGL((k_gemm_valu<RPW, WPL>), dim3((unsigned)(ctiles * rtiles)), dim3(256), 0, s, g.A, g.lda, g.B,
                       g.ldb, g.Cold, g.ldco, g.C, g.ldc, g.D, g.ldd, g.M, g.K, g.N, g.changed);
  } else {
    constexpr int WPL = 1;
    const i64 ctiles = 1;
    const i64 rtiles = (g.M + 4 * RPW - 1) / (4 * RPW);
    hipLaunchKernelGGL((k_gemm_valu<RPW, WPL>), dim3((unsigned)(ctiles * rtiles)), dim3(256), 0, s, g.A, g.lda, g.B,
                       g.ldb, g.Cold, g.ldco, g.C, g.ldc, g.D, g.ldd, g.M, g.K, g.N, g.changed);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_mfma(const GemmArgs& g, const u64* BT, i64 ldbt, hipStream_t s) {
  (void)BT;
  (void)ldbt;
  return launch_gemm_valu(g, s);
}

}  // namespace bmlp
