// The bit-packed (VALU) product tile, shared by the single-product kernel and
// the batched round kernel.
//
// Row-OR formulation of the Boolean product (Section 2): C[i,:] |= B[k,:] for
// every set bit A[i,k].  A workgroup of 256 threads owns a tile of 4*RPW rows
// x 64*WPL words of the output.  Wave w owns rows row0 .. row0+RPW-1 (row0 is
// wave-uniform), lane l owns words w0 + l + 64*j (j < WPL).  For each word kw
// of k (64 values of k) the workgroup stages B[64 kw .. 64 kw + 63, tile words]
// in LDS; the A word of each of the wave's rows is wave-uniform, so the AND
// mask for (i, k) is one scalar value and each lane spends one v_and_or_b32 per
// 32 bit-MACs.  Words of k for which no row of the tile has a set bit are
// skipped, B staging included (sparse A).
#pragma once
#include "bmlp_internal.h"

namespace bmlp {

// a wave-uniform 64-bit value moved to scalar registers (each half zero-extended)
__device__ __forceinline__ u64 uniform64(u64 v) {
  const u32 lo = (u32)__builtin_amdgcn_readfirstlane((int)(u32)v);
  const u32 hi = (u32)__builtin_amdgcn_readfirstlane((int)(u32)(v >> 32));
  return ((u64)hi << 32) | (u64)lo;
}

// all-ones when bit `b` of the wave-uniform word x is set, else zero
__device__ __forceinline__ u32 bit_mask(u32 x, int b) { return (u32)(((int)(x << (31 - b))) >> 31); }

// acc | (b & m) as one v_and_or_b32 (m is a scalar operand)
__device__ __forceinline__ u32 and_or(u32 b, u32 m, u32 acc) {
  u32 r;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(b), "s"(m), "v"(acc));
  return r;
}

// acc |= A[row0 .. row0+RPW, k words kw_begin..kw_end) . B[those k, w0 .. w0 + 64 WPL)
// All threads of the workgroup must call it with the same kw range and w0.  Returns whether any word
// of k had a set bit in a row of the tile (the same answer in every thread of the workgroup).
template <int RPW, int WPL>
__device__ __forceinline__ bool valu_tile_accumulate(const u64* __restrict__ A, i64 lda, const u64* __restrict__ B,
                                                     i64 ldb, i64 M, i64 K, i64 nw, i64 row0, i64 w0, i64 kw_begin,
                                                     i64 kw_end, u64 (*Bs)[64 * WPL], u32 (&acc)[RPW][WPL][2]) {
  constexpr int TW = 64 * WPL;
  const int lane = threadIdx.x & 63;
  bool worked = false;  // some word of k had a set bit in some row of the tile (workgroup-uniform)
  for (i64 kw = kw_begin; kw < kw_end; ++kw) {
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
    worked = true;
    // stage the 64 x TW chunk of B: every thread's loads are issued before any is waited for.
    // They are clamped into the matrix, so they need no guard (words outside it are stored as
    // zero), and addressed by 32-bit offsets from the chunk's first row.
    constexpr int kPer = 64 * TW / 256;
    const u64* Bk = B + kw * 64 * ldb;
    const int klast = (int)(K - 1 - kw * 64 < 63 ? K - 1 - kw * 64 : 63);  // last row of the chunk in B
    const int clast = (int)(nw - 1 - w0 < TW - 1 ? nw - 1 - w0 : TW - 1);   // last column of the tile in B
    u64 st[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int idx = threadIdx.x + 256 * i;
      const int r = idx / TW, c = idx % TW;
      const u32 off = (u32)(r < klast ? r : klast) * (u32)ldb + (u32)w0 + (u32)(c < clast ? c : clast);
      st[i] = Bk[off];
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int idx = threadIdx.x + 256 * i;
      const int r = idx / TW, c = idx % TW;
      Bs[r][c] = (r <= klast && c <= clast) ? st[i] : 0ull;
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
  return worked;
}

// C = Cold | acc for the tile (D = C & ~Cold when D is given); returns whether
// any word of this lane changed and adds the number of new bits to *pop.
template <int RPW, int WPL>
__device__ __forceinline__ int valu_tile_store(const u32 (&acc)[RPW][WPL][2], const u64* __restrict__ Cold, i64 ldco,
                                               u64* __restrict__ C, i64 ldc, u64* __restrict__ D, i64 ldd, i64 M,
                                               i64 nw, i64 row0, i64 w0, u32* pop = nullptr) {
  const int lane = threadIdx.x & 63;
  int ch = 0;
  u32 cnt = 0;
  // C_old is read first, all RPW x WPL words at once (clamped to the matrix, unguarded, so that the
  // loads overlap instead of each being waited for behind its bounds check)
  u64 old[RPW][WPL];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const i64 rc = row0 + r < M ? row0 + r : M - 1;
#pragma unroll
    for (int wl = 0; wl < WPL; ++wl) {
      const i64 w = w0 + lane + 64 * wl;
      old[r][wl] = Cold ? Cold[rc * ldco + (w < nw ? w : nw - 1)] : 0ull;
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const i64 row = row0 + r;
    if (row >= M) break;
#pragma unroll
    for (int wl = 0; wl < WPL; ++wl) {
      const i64 w = w0 + lane + 64 * wl;
      if (w < nw) {
        const u64 v = (((u64)acc[r][wl][1] << 32) | (u64)acc[r][wl][0]) | old[r][wl];
        C[row * ldc + w] = v;
        if (D) D[row * ldd + w] = v & ~old[r][wl];
        ch |= (v != old[r][wl]);
        cnt += (u32)__popcll(v & ~old[r][wl]);
      }
    }
  }
  if (pop) *pop += cnt;
  return ch;
}

// adds the wave's sum of `v` into *counter (one atomic per wave)
__device__ __forceinline__ void wave_count(u32 v, unsigned long long* counter) {
  if (!counter) return;
  u64 s = v;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(counter, (unsigned long long)s);
}

// The workgroup's sum of `v` into *counter and, when some thread passes any != 0, *changed |= 1: one device
// atomic per workgroup and target, the waves' parts meeting in `slot` (LDS) first.  Same-address device
// atomics are serialised, so a launch of many short waves that each add to one counter (16,384 waves for a
// squaring of 16,384 rows by gathers) waits for them.  Every thread of the workgroup calls it, after its
// last use of `slot`; counter and changed may be null.
template <int Waves>
__device__ __forceinline__ void block_counts(u32 v, int any, unsigned long long* counter, u32* changed,
                                             unsigned long long (&slot)[Waves][2]) {
  if (!counter && !changed) return;  // the same in every thread
  u64 s = v;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const u64 bal = __ballot(any);
  if ((threadIdx.x & 63) == 0) {
    slot[threadIdx.x >> 6][0] = s;
    slot[threadIdx.x >> 6][1] = bal != 0ull ? 1ull : 0ull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 t = 0, c = 0;
#pragma unroll
    for (int i = 0; i < Waves; ++i) {
      t += slot[i][0];
      c |= slot[i][1];
    }
    if (counter && t) atomicAdd(counter, (unsigned long long)t);
    if (changed && c) atomicOr(changed, 1u);
  }
}

}  // namespace bmlp
