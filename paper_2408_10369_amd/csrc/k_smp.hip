// Selective matrix product (BMLP-SMP, Section 3.3 Eq. 5 and Algorithm 2),
// sparse-frontier arm.  One workgroup owns one query row r and runs the whole
// fixpoint for it in a single launch, with three n-bit bitmaps in LDS:
//
//   vis : nodes reached so far by paths of length >= 1 from the row's sources
//   fr  : the frontier (bits new in the last round; the sources at the start)
//   nxt : successors of the frontier in the current round
//
// Each round is one semi-naive step of the selection: nxt = fr . R1,
// fr = nxt & ~vis, vis |= fr.  It stops when fr is empty, which is the
// "v* = v'" test of Algorithm 2 (the iterates are monotone).  Starting the
// frontier at the sources and never marking them visited up front yields
// exactly v R1+, so no final product with R1 is needed; the reflexive mode
// adds the sources at the end (v R1*).
//
// Frontier nodes of low out-degree are expanded by the thread that finds them
// through the CSR successor list (LDS atomic ORs).  High-degree nodes are
// queued and expanded by the whole workgroup, either through CSR or, when the
// node's row is dense, by OR-ing its bit row of R1 word by word.
#include "bmlp_internal.h"
#include "valu_tile.h"

namespace bmlp {

namespace {

constexpr int kSmpThreads = 256;
constexpr int kHubDeg = 48;       // expand cooperatively above this out-degree
constexpr int kHubCap = 512;      // LDS queue of cooperative nodes per round
constexpr i64 kMaxLdsWords = 6144;  // 3 bitmaps x 2048 words = 48 KiB (n <= 131072)

// SLOTS: unvisited nodes a thread checks at once in a bottom-up round.  Eight hide the latency of the
// in-edge loads when few rows share the launch; with many rows the registers they take would cut the
// workgroups a CU holds (97 against 54 VGPRs), so one is used there.
template <int SLOTS>
__global__ void __launch_bounds__(kSmpThreads)
k_smp_rows(const u64* __restrict__ V, i64 ldv, i64 k, const i64* __restrict__ rp, const int32_t* __restrict__ ci,
           const i64* __restrict__ rpt, const int32_t* __restrict__ cit, const u64* __restrict__ R, i64 ldr, i64 n,
           int reflexive, u64* __restrict__ out, i64 ldo, u32* __restrict__ iters_max) {
  extern __shared__ u64 smem[];
  __shared__ int32_t hubs[kHubCap];
  __shared__ int nhubs;
  __shared__ u32 cnt[2][2];  // by round parity: frontier size, visited size
  const i64 nw = (n + 63) >> 6;
  u64* vis = smem;
  u64* fr = smem + nw;
  u64* nxt = smem + 2 * nw;
  u32* nxt32 = (u32*)nxt;
  const int t = threadIdx.x;
  const int lane = t & 63;
  // columns >= n never enter a bitmap, whatever the padding bits of the inputs hold
  const u64 last_mask = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
  const double davg = (double)rp[n] / (double)(n > 0 ? n : 1);  // mean out-degree

  for (i64 row = blockIdx.x; row < k; row += gridDim.x) {
    if (t < 4) cnt[t >> 1][t & 1] = 0u;
    if (t == 0) nhubs = 0;
    __syncthreads();
    u32 nf0 = 0;
    for (i64 w = t; w < nw; w += kSmpThreads) {
      vis[w] = 0ull;
      // V null: the rows of the identity (row i starts from node i), so the answers are the rows of R1+
      const u64 f = V ? V[row * ldv + w] & (w == nw - 1 ? last_mask : ~0ull)
                      : (w == (row >> 6) && row < n ? 1ull << (row & 63) : 0ull);
      fr[w] = f;
      nxt[w] = 0ull;
      nf0 += (u32)__popcll(f);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nf0 += __shfl_xor(nf0, off, 64);
    if (lane == 0 && nf0) atomicAdd(&cnt[0][0], nf0);
    __syncthreads();
    u32 rounds = 0;
    for (;;) {
      const int par = (int)(rounds & 1u);
      ++rounds;
      // direction of this round (the same in every thread): top-down visits the out-edges of the
      // frontier, bottom-up the in-edges of the unvisited nodes until one comes from the frontier
      const double nf = (double)cnt[par][0], nu = (double)n - (double)cnt[par][1];
      const bool bottom_up = rpt && nf * davg > nu * fmin(davg, (double)n / fmax(nf, 1.0));
      if (t < 2) cnt[par ^ 1][t] = 0u;  // read above; the syncs below order it before the next counts
      if (bottom_up) {
        for (i64 w = t; w < nw; w += kSmpThreads) {
          u64 cand = ~vis[w] & (w == nw - 1 ? last_mask : ~0ull);
          u64 found = 0ull;
          // SLOTS candidates in flight: slot q scans the in-edges [se, sx) of node 64 w + sb until one
          // comes from the frontier or the list ends, then takes the next candidate, so that the
          // thread's in-edge loads overlap instead of forming one chain
          int sb[SLOTS];
          i64 se[SLOTS], sx[SLOTS];
#pragma unroll
          for (int q = 0; q < SLOTS; ++q) {
            sb[q] = -1;
            se[q] = sx[q] = 0;
            if (cand) {
              const int b = __ffsll((unsigned long long)cand) - 1;
              cand &= cand - 1;
              sb[q] = b;
              se[q] = rpt[w * 64 + b];
              sx[q] = rpt[w * 64 + b + 1];
            }
          }
          for (;;) {
            int32_t u[SLOTS];
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) u[q] = (sb[q] >= 0 && se[q] < sx[q]) ? cit[se[q]] : -1;
            bool busy = false;
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) {
              if (sb[q] < 0) continue;
              bool done = true;  // a node without (more) in-edges is not reached this round
              if (u[q] >= 0) {
                if ((fr[u[q] >> 6] >> (u[q] & 63)) & 1ull) found |= 1ull << sb[q];
                else done = ++se[q] >= sx[q];
              }
              if (done) {
                sb[q] = -1;
                if (cand) {
                  const int b = __ffsll((unsigned long long)cand) - 1;
                  cand &= cand - 1;
                  sb[q] = b;
                  se[q] = rpt[w * 64 + b];
                  sx[q] = rpt[w * 64 + b + 1];
                }
              }
              busy |= sb[q] >= 0;
            }
            if (!busy) break;
          }
          nxt[w] = found;
        }
        __syncthreads();
      } else {
        // expand the frontier
        for (i64 w = t; w < nw; w += kSmpThreads) {
          u64 x = fr[w];
          while (x) {
            const int b = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            const i64 u = w * 64 + b;
            const i64 e0 = rp[u], e1 = rp[u + 1];
            if (e1 - e0 > kHubDeg) {
              const int slot = atomicAdd(&nhubs, 1);
              if (slot < kHubCap) {
                hubs[slot] = (int32_t)u;
                continue;
              }
            }
            for (i64 e = e0; e < e1; ++e) {
              const int32_t v = ci[e];
              atomicOr(&nxt32[v >> 5], 1u << (v & 31));
            }
          }
        }
        __syncthreads();
        const int nh = nhubs < kHubCap ? nhubs : kHubCap;  // the same in every thread after the barrier
        // hubs whose bit row is denser than their successor list (out-degree > nw / 2) are ORed from R, eight
        // rows per pass with their loads in flight together; the others are expanded through CSR, a wave each
        for (int h0 = 0; h0 < nh; h0 += 8) {
          i64 dense[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            dense[q] = -1;
            if (h0 + q < nh) {
              const i64 u = hubs[h0 + q];
              if (R && (rp[u + 1] - rp[u]) * 2 > nw) dense[q] = u;
            }
          }
          for (i64 w = t; w < nw; w += kSmpThreads) {
            u64 x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = dense[q] >= 0 ? R[dense[q] * ldr + w] : 0ull;
            u64 acc = 0ull;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc |= x[q];
            if (acc) {
              atomicOr(&nxt32[2 * w], (u32)acc);
              atomicOr(&nxt32[2 * w + 1], (u32)(acc >> 32));
            }
          }
          // each wave expands two of the batch's CSR hubs, its lanes over the successor list
          for (int q = t >> 6; q < 8; q += kSmpThreads / 64) {
            if (h0 + q >= nh || dense[q] >= 0) continue;
            const i64 u = hubs[h0 + q];
            const i64 e1 = rp[u + 1];
            for (i64 e = rp[u] + lane; e < e1; e += 64) {
              const int32_t v = ci[e];
              atomicOr(&nxt32[v >> 5], 1u << (v & 31));
            }
          }
        }
        if (nh > 0) __syncthreads();
      }
      // fr = nxt & ~vis ; vis |= fr ; nxt = 0
      int any = 0;
      u32 lf = 0, lv = 0;
      for (i64 w = t; w < nw; w += kSmpThreads) {
        const u64 nv = nxt[w] & ~vis[w] & (w == nw - 1 ? last_mask : ~0ull);
        const u64 vv = vis[w] | nv;
        vis[w] = vv;
        fr[w] = nv;
        nxt[w] = 0ull;
        any |= (nv != 0ull);
        lf += (u32)__popcll(nv);
        lv += (u32)__popcll(vv);
      }
      if (rpt) {  // the counts only steer the direction
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          lf += __shfl_xor(lf, off, 64);
          lv += __shfl_xor(lv, off, 64);
        }
        if (lane == 0) {
          if (lf) atomicAdd(&cnt[par ^ 1][0], lf);
          if (lv) atomicAdd(&cnt[par ^ 1][1], lv);
        }
      }
      if (t == 0) nhubs = 0;
      if (!__syncthreads_or(any)) break;
      if ((i64)rounds > n + 1) break;  // unreachable for a correct monotone iteration
    }
    for (i64 w = t; w < nw; w += kSmpThreads) {
      u64 v = vis[w];
      if (reflexive)
        v |= V ? V[row * ldv + w] & (w == nw - 1 ? last_mask : ~0ull) : (w == (row >> 6) ? 1ull << (row & 63) : 0ull);
      out[row * ldo + w] = v;
    }
    for (i64 w = nw + t; w < ldo; w += kSmpThreads) out[row * ldo + w] = 0ull;
    if (t == 0 && iters_max) atomicMax(iters_max, rounds);
    __syncthreads();
  }
}

// One round of the semi-naive selection for every query row, state in global
// memory (the same round as one dense product): nxt = fr[r] . R1 by CSR
// expansion in LDS, fr_out[r] = nxt & ~vis[r], vis[r] |= fr_out[r].  Rows with
// an empty frontier only write their empty fr_out row.  Sets *changed and adds
// the number of new bits to *newbits.  Runs only if *pred == pred_val (when
// pred is given), so that the host can queue both arms of a round and let the
// device-side choice decide.
__global__ void __launch_bounds__(kSmpThreads)
k_smp_round(const u64* __restrict__ fr, u64* __restrict__ fr_out, i64 ldf, u64* __restrict__ vis, i64 ldvis, i64 k,
            const i64* __restrict__ rp, const int32_t* __restrict__ ci, const u64* __restrict__ R, i64 ldr, i64 n,
            u32* __restrict__ changed, unsigned long long* __restrict__ newbits, const u32* __restrict__ pred,
            u32 pred_val) {
  extern __shared__ u64 smem[];
  __shared__ int32_t hubs[kHubCap];
  __shared__ int nhubs;
  if (pred && *pred != pred_val) return;
  const i64 nw = (n + 63) >> 6;
  u64* nxt = smem;
  u32* nxt32 = (u32*)nxt;
  const int t = threadIdx.x;
  const u64 last_mask = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
  u32 cnt = 0;
  int any = 0;
  for (i64 row = blockIdx.x; row < k; row += gridDim.x) {
    for (i64 w = t; w < nw; w += kSmpThreads) nxt[w] = 0ull;
    if (t == 0) nhubs = 0;
    __syncthreads();
    for (i64 w = t; w < nw; w += kSmpThreads) {
      u64 x = fr[row * ldf + w] & (w == nw - 1 ? last_mask : ~0ull);
      while (x) {
        const int b = __ffsll((unsigned long long)x) - 1;
        x &= x - 1;
        const i64 u = w * 64 + b;
        const i64 e0 = rp[u], e1 = rp[u + 1];
        if (e1 - e0 > kHubDeg) {
          const int slot = atomicAdd(&nhubs, 1);
          if (slot < kHubCap) {
            hubs[slot] = (int32_t)u;
            continue;
          }
        }
        for (i64 e = e0; e < e1; ++e) {
          const int32_t v = ci[e];
          atomicOr(&nxt32[v >> 5], 1u << (v & 31));
        }
      }
    }
    __syncthreads();
    const int nh = nhubs < kHubCap ? nhubs : kHubCap;
    for (int h = 0; h < nh; ++h) {
      const i64 u = hubs[h];
      const i64 e0 = rp[u], e1 = rp[u + 1];
      if (R && (e1 - e0) * 2 > nw) {
        for (i64 w = t; w < nw; w += kSmpThreads) {
          const u64 x = R[u * ldr + w];
          if (x) {
            atomicOr(&nxt32[2 * w], (u32)x);
            atomicOr(&nxt32[2 * w + 1], (u32)(x >> 32));
          }
        }
      } else {
        for (i64 e = e0 + t; e < e1; e += kSmpThreads) {
          const int32_t v = ci[e];
          atomicOr(&nxt32[v >> 5], 1u << (v & 31));
        }
      }
    }
    __syncthreads();
    for (i64 w = t; w < nw; w += kSmpThreads) {
      const u64 old = vis[row * ldvis + w];
      const u64 nv = nxt[w] & ~old & (w == nw - 1 ? last_mask : ~0ull);
      if (nv) {
        vis[row * ldvis + w] = old | nv;
        cnt += (u32)__popcll(nv);
        any = 1;
      }
      fr_out[row * ldf + w] = nv;
    }
    __syncthreads();
  }
  __shared__ unsigned long long cslot[kSmpThreads / 64][2];
  block_counts<kSmpThreads / 64>(cnt, any, newbits, changed, cslot);
}

// Selection read off a closure: out[r] = OR of C[u, :] over the set bits u of V[r] (V[r] R1+ when C
// is R1+; reflexive adds V[r] itself).  One workgroup per row.  Thread t counts the set bits of its
// contiguous share of V[r], a workgroup prefix scan numbers them, and the source rows are listed in
// LDS in passes of 1,024 and OR-ed, each a coalesced row of C, into the answer held in registers
// (thread t owns words t, t + 256, ...; n <= 131,072).  The answer of row r goes to output row
// row_map[r] (r without a map) and starts from zero, from V[r] (init 1) or from the output row's
// current content (init 2); the bits added to those starting rows are counted into *newbits.
constexpr int kGatherWords = 2048;

__global__ void __launch_bounds__(256)
k_gather_rows(const u64* __restrict__ V, i64 ldv, i64 k, const u64* __restrict__ Cl, i64 ldc, i64 n, int init,
              u64* __restrict__ out, i64 ldo, const int32_t* __restrict__ row_map,
              unsigned long long* __restrict__ newbits, const u32* __restrict__ pred, u32 pred_val) {
  __shared__ int32_t srcs[1024];
  __shared__ int scan[256];
  if (pred && *pred != pred_val) return;
  const i64 nw = (n + 63) >> 6;
  const u64 last_mask = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
  const int t = threadIdx.x;
  const i64 chunk = (nw + 255) / 256;
  const i64 wb = t * chunk, we = (wb + chunk < nw) ? wb + chunk : nw;
  u32 added = 0;  // bits of the answers not in their starting rows
  for (i64 row = blockIdx.x; row < k; row += gridDim.x) {
    const i64 orow = row_map ? (i64)row_map[row] : row;
    u64 acc[kGatherWords / 256], start[kGatherWords / 256];
#pragma unroll
    for (int j = 0; j < kGatherWords / 256; ++j) {
      const i64 w = t + 256 * j;
      u64 a = 0ull;
      if (w < nw && init == 1) a = V[row * ldv + w] & (w == nw - 1 ? last_mask : ~0ull);
      if (w < nw && init == 2) a = out[orow * ldo + w];
      acc[j] = a;
      start[j] = a;
    }
    int cnt = 0;
    for (i64 w = wb; w < we; ++w) cnt += __popcll(V[row * ldv + w] & (w == nw - 1 ? last_mask : ~0ull));
    scan[t] = cnt;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int v = t >= off ? scan[t - off] : 0;
      __syncthreads();
      scan[t] += v;
      __syncthreads();
    }
    const int total = scan[255];
    const int first = scan[t] - cnt;  // global index of this thread's first source
    __syncthreads();
    for (int base = 0; base < total; base += 1024) {
      int idx = first;
      for (i64 w = wb; w < we && idx < base + 1024; ++w) {
        u64 x = V[row * ldv + w] & (w == nw - 1 ? last_mask : ~0ull);
        while (x) {
          const int b = __ffsll((unsigned long long)x) - 1;
          x &= x - 1;
          if (idx >= base && idx < base + 1024) srcs[idx - base] = (int32_t)(w * 64 + b);
          ++idx;
        }
      }
      __syncthreads();
      const int c = (total - base) < 1024 ? (total - base) : 1024;
      // eight source rows per step, so that eight independent loads per word are in flight
      int i = 0;
      for (; i + 8 <= c; i += 8) {
        i64 u[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) u[q] = srcs[i + q];
#pragma unroll
        for (int j = 0; j < kGatherWords / 256; ++j) {
          const i64 w = t + 256 * j;
          if (w < nw) {
            u64 x = 0ull;
#pragma unroll
            for (int q = 0; q < 8; ++q) x |= Cl[u[q] * ldc + w];
            acc[j] |= x;
          }
        }
      }
      for (; i < c; ++i) {
        const i64 u = srcs[i];
#pragma unroll
        for (int j = 0; j < kGatherWords / 256; ++j) {
          const i64 w = t + 256 * j;
          if (w < nw) acc[j] |= Cl[u * ldc + w];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kGatherWords / 256; ++j) {
      const i64 w = t + 256 * j;
      if (w < nw) {
        out[orow * ldo + w] = acc[j];
        added += (u32)__popcll(acc[j] & ~start[j]);
      }
    }
    for (i64 w = nw + t; w < ldo; w += 256) out[orow * ldo + w] = 0ull;
    __syncthreads();
  }
  __shared__ unsigned long long cslot[4][2];
  block_counts<4>(added, 0, newbits, nullptr, cslot);
}

// The same gather with one wave per row, for n <= 16,384 (lane l owns words l + 64 j, j < WPL): no
// workgroup scan, and the set bits of the row are walked in batches of eight (across its words), so
// that eight source-row loads per word are in flight at a time.
//
// A wave walks a source row in about 170 ns, so one row with thousands of set bits would hold the whole
// launch up.  With an overflow queue (qe != nullptr) a row with more than `piece` set bits walks only
// its first `piece` and queues the rest as pieces (row, j) of `piece` bits each (a multiple of 8), for
// k_gather_rows_q, launched after this kernel, to OR into the row with 64-bit atomics.
constexpr int kMinPiece = 64;

// The piece size: the host's, or -- with a device count of V's set bits -- twice the mean row of V's `rows`
// rows, at least kMinPiece, at most 2^24, a multiple of 8 (the host's rule, sized()).
__device__ __forceinline__ int gather_piece(int piece, const unsigned long long* __restrict__ bits, i64 rows) {
  if (!bits) return piece;
  const unsigned long long mean = *bits / (unsigned long long)(rows > 0 ? rows : 1);
  unsigned long long p = 2ull * mean;
  if (p < (unsigned long long)kMinPiece) p = kMinPiece;
  if (p > (1ull << 24)) p = 1ull << 24;
  return (int)((p + 7ull) / 8ull * 8ull);
}

template <int WPL>
__global__ void __launch_bounds__(256)
k_gather_rows_w(const u64* __restrict__ V, i64 ldv, i64 k, const u64* __restrict__ Cl, i64 ldc, i64 n, int init,
                u64* __restrict__ out, i64 ldo, const int32_t* __restrict__ row_map,
                unsigned long long* __restrict__ newbits, int2* __restrict__ qe, unsigned long long* __restrict__ qn,
                i64 qcap, int piece_arg, const unsigned long long* __restrict__ vbits, const u32* __restrict__ pred,
                u32 pred_val) {
  if (pred && *pred != pred_val) return;  // another kernel serves this squaring
  const int piece = gather_piece(piece_arg, vbits, k);
  const int lane = threadIdx.x & 63;
  const i64 wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const i64 nwaves = (i64)gridDim.x * 4;
  const i64 nw = (n + 63) >> 6;
  const u64 last_mask = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
  u32 added = 0;  // bits of the answers not in their starting rows
  for (i64 row = wave; row < k; row += nwaves) {
    const i64 orow = row_map ? (i64)row_map[row] : row;
    u64 vr[WPL], acc[WPL], start[WPL], nz[WPL];
#pragma unroll
    for (int j = 0; j < WPL; ++j) {
      const i64 w = lane + 64 * j;
      vr[j] = w < nw ? V[row * ldv + w] & (w == nw - 1 ? last_mask : ~0ull) : 0ull;
      u64 a = 0ull;
      if (w < nw && init == 1) a = vr[j];
      if (w < nw && init == 2) a = out[orow * ldo + w];
      acc[j] = a;
      start[j] = a;
      nz[j] = __ballot(vr[j] != 0ull);  // words of the row with set bits (wave-uniform)
    }
    int limit = 1 << 30;  // sources this wave walks
    if (qe) {
      u32 c = 0;
#pragma unroll
      for (int j = 0; j < WPL; ++j) c += (u32)__popcll(vr[j]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
      if (c > (u32)piece) {
        const u32 extra = (c - 1) / (u32)piece;  // pieces after the first
        unsigned long long base = 0ull;
        if (lane == 0) base = atomicAdd(qn, (unsigned long long)extra);
        base = uniform64(base);
        for (u32 i = lane; i < extra; i += 64) {
          const unsigned long long slot = base + i;
          if ((i64)slot < qcap) qe[slot] = make_int2((int)row, (int)(i + 1));
        }
        limit = piece;
      }
    }
    // The walk over the row's set bits is wave-uniform: its state (word, remaining bits, sources)
    // lives in scalar registers, so the sources address their rows from scalar bases.
    int w = 0;
    u64 x = 0ull;
    for (int walked = 0; walked < limit; walked += 8) {
      int src[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
#pragma unroll
        for (int j = 0; j < WPL; ++j) {
          if (!x && nz[j]) {
            const int b = __ffsll((unsigned long long)nz[j]) - 1;
            nz[j] &= nz[j] - 1;
            w = 64 * j + b;
            x = uniform64(__shfl(vr[j], b, 64));
          }
        }
        src[q] = -1;
        if (x) {
          src[q] = 64 * w + (__ffsll((unsigned long long)x) - 1);
          x &= x - 1;
        }
      }
      if (src[0] < 0) break;
      // Every load is issued unguarded so that all 8 x WPL of them are in flight together: a
      // missing source repeats src[0] and is masked out, and a lane past the row's last word
      // re-reads that word and drops it.
      const u64* rowp[8];
      u64 keep[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        keep[q] = src[q] >= 0 ? ~0ull : 0ull;
        rowp[q] = Cl + (i64)(src[q] >= 0 ? src[q] : src[0]) * ldc;
      }
      u64 t[WPL][8];
#pragma unroll
      for (int j = 0; j < WPL; ++j) {
        const int ww = lane + 64 * j;
        const int wc = ww < nw ? ww : (int)nw - 1;
#pragma unroll
        for (int q = 0; q < 8; ++q) t[j][q] = rowp[q][wc];
      }
#pragma unroll
      for (int j = 0; j < WPL; ++j) {
        u64 v = 0ull;
#pragma unroll
        for (int q = 0; q < 8; ++q) v |= t[j][q] & keep[q];
        if (lane + 64 * j < nw) acc[j] |= v;
      }
    }
#pragma unroll
    for (int j = 0; j < WPL; ++j) {
      const i64 ww = lane + 64 * j;
      if (ww < nw) {
        out[orow * ldo + ww] = acc[j];
        added += (u32)__popcll(acc[j] & ~start[j]);
      }
    }
    for (i64 ww = nw + lane; ww < ldo; ww += 64) out[orow * ldo + ww] = 0ull;
  }
  __shared__ unsigned long long cslot[4][2];
  block_counts<4>(added, 0, newbits, nullptr, cslot);
}

// The queued pieces of the heavy rows: piece (row, j) walks the set bits numbered [p j, p j + p) of
// V[row] in word order and ORs the gathered rows into out[map(row)] with 64-bit atomics; the value each
// atomic returns tells which of its bits are new, so *newbits stays exact.  The rows already hold their
// starting value and first piece (k_gather_rows_w, launched before).
template <int WPL>
__global__ void __launch_bounds__(256)
k_gather_rows_q(const u64* __restrict__ V, i64 ldv, i64 k, const u64* __restrict__ Cl, i64 ldc, i64 n,
                u64* __restrict__ out, i64 ldo, const int32_t* __restrict__ row_map, const int2* __restrict__ qe,
                const unsigned long long* __restrict__ qn, i64 qcap, int piece_arg,
                const unsigned long long* __restrict__ vbits, unsigned long long* __restrict__ newbits,
                const u32* __restrict__ pred, u32 pred_val) {
  if (pred && *pred != pred_val) return;
  const int piece = gather_piece(piece_arg, vbits, k);  // the same as k_gather_rows_w's
  const int lane = threadIdx.x & 63;
  const i64 wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const i64 nwaves = (i64)gridDim.x * 4;
  const i64 nw = (n + 63) >> 6;
  const u64 last_mask = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
  const i64 queued = (i64)*qn;
  const i64 cnt = queued < qcap ? queued : qcap;
  u32 added = 0;
  for (i64 e = wave; e < cnt; e += nwaves) {
    const int2 pc = qe[e];
    const i64 row = pc.x;
    const i64 orow = row_map ? (i64)row_map[row] : row;
    const i64 skip = (i64)pc.y * piece;
    u64 vr[WPL], acc[WPL], nz[WPL];
    i64 before = 0;  // set bits of the row in the blocks before j
#pragma unroll
    for (int j = 0; j < WPL; ++j) {
      const i64 w = lane + 64 * j;
      u64 v = w < nw ? V[row * ldv + w] & (w == nw - 1 ? last_mask : ~0ull) : 0ull;
      // drop the set bits numbered below skip: inclusive scan of the popcounts across the lanes
      const u32 c = (u32)__popcll(v);
      u32 incl = c;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const u32 y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
      }
      const i64 drop = skip - (before + (i64)(incl - c));
      if (drop >= (i64)c) v = 0ull;
      else
        for (i64 d = 0; d < drop; ++d) v &= v - 1;
      before += (i64)__shfl(incl, 63, 64);
      vr[j] = v;
      acc[j] = 0ull;
      nz[j] = __ballot(v != 0ull);
    }
    int w = 0;
    u64 x = 0ull;
    for (int walked = 0; walked < piece; walked += 8) {
      int src[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
#pragma unroll
        for (int j = 0; j < WPL; ++j) {
          if (!x && nz[j]) {
            const int b = __ffsll((unsigned long long)nz[j]) - 1;
            nz[j] &= nz[j] - 1;
            w = 64 * j + b;
            x = uniform64(__shfl(vr[j], b, 64));
          }
        }
        src[q] = -1;
        if (x) {
          src[q] = 64 * w + (__ffsll((unsigned long long)x) - 1);
          x &= x - 1;
        }
      }
      if (src[0] < 0) break;
      const u64* rowp[8];
      u64 keep[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        keep[q] = src[q] >= 0 ? ~0ull : 0ull;
        rowp[q] = Cl + (i64)(src[q] >= 0 ? src[q] : src[0]) * ldc;
      }
      u64 t[WPL][8];
#pragma unroll
      for (int j = 0; j < WPL; ++j) {
        const int ww = lane + 64 * j;
        const int wc = ww < nw ? ww : (int)nw - 1;
#pragma unroll
        for (int q = 0; q < 8; ++q) t[j][q] = rowp[q][wc];
      }
#pragma unroll
      for (int j = 0; j < WPL; ++j) {
        u64 v = 0ull;
#pragma unroll
        for (int q = 0; q < 8; ++q) v |= t[j][q] & keep[q];
        if (lane + 64 * j < nw) acc[j] |= v;
      }
    }
#pragma unroll
    for (int j = 0; j < WPL; ++j) {
      const i64 ww = lane + 64 * j;
      if (ww < nw && acc[j]) {
        const u64 old = atomicOr((unsigned long long*)&out[orow * ldo + ww], (unsigned long long)acc[j]);
        added += (u32)__popcll(acc[j] & ~old);
      }
    }
  }
  __shared__ unsigned long long cslot[4][2];
  block_counts<4>(added, 0, newbits, nullptr, cslot);
}

}  // namespace

i64 smp_rows_max_n() { return (kMaxLdsWords / 3) * 64; }

i64 gather_rows_max_n() { return (i64)kGatherWords * 64; }

i64 gather_queue_capacity(i64 k, i64 n) { return k * ((n + kMinPiece - 1) / kMinPiece); }

hipError_t launch_gather_rows(const u64* V, i64 ldv, i64 k, const u64* Cl, i64 ldc, i64 n, int init, u64* out,
                              i64 ldo, hipStream_t s, const int32_t* row_map, unsigned long long* newbits,
                              const GatherQueue* q, const u32* pred, u32 pred_val) {
  if (k <= 0) return hipSuccess;
  const i64 nw = words_for(n);
  if (nw > kGatherWords) return hipErrorInvalidValue;
  if (nw <= 256) {
    const bool queued = q && q->e && q->n && q->cap >= gather_queue_capacity(k, n);
    int2* qe = queued ? q->e : nullptr;
    unsigned long long* qn = queued ? q->n : nullptr;
    const i64 qcap = queued ? q->cap : 0;
    const int piece = queued ? (std::max(q->piece, kMinPiece) + 7) / 8 * 8 : kMinPiece;
    const unsigned long long* vbits = queued ? q->bits : nullptr;
    if (queued) {
      const hipError_t e = launch_fill_zero((u64*)qn, 1, s);
      if (e != hipSuccess) return e;
    }
    const i64 blocks = (k + 3) / 4;
    const unsigned grid = (unsigned)(blocks < 16384 ? blocks : 16384);
    if (nw <= 64)
      hipLaunchKernelGGL(k_gather_rows_w<1>, dim3(grid), dim3(256), 0, s, V, ldv, k, Cl, ldc, n, init, out, ldo,
                         row_map, newbits, qe, qn, qcap, piece, vbits, pred, pred_val);
    else if (nw <= 128)
      hipLaunchKernelGGL(k_gather_rows_w<2>, dim3(grid), dim3(256), 0, s, V, ldv, k, Cl, ldc, n, init, out, ldo,
                         row_map, newbits, qe, qn, qcap, piece, vbits, pred, pred_val);
    else
      hipLaunchKernelGGL(k_gather_rows_w<4>, dim3(grid), dim3(256), 0, s, V, ldv, k, Cl, ldc, n, init, out, ldo,
                         row_map, newbits, qe, qn, qcap, piece, vbits, pred, pred_val);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !queued) return e;
    // the pieces: their number is known on the device only, so a fixed grid strides over them
    const unsigned qgrid = grid < 2048 ? grid : 2048;
    if (nw <= 64)
      hipLaunchKernelGGL(k_gather_rows_q<1>, dim3(qgrid), dim3(256), 0, s, V, ldv, k, Cl, ldc, n, out, ldo, row_map,
                         qe, qn, qcap, piece, vbits, newbits, pred, pred_val);
    else if (nw <= 128)
      hipLaunchKernelGGL(k_gather_rows_q<2>, dim3(qgrid), dim3(256), 0, s, V, ldv, k, Cl, ldc, n, out, ldo, row_map,
                         qe, qn, qcap, piece, vbits, newbits, pred, pred_val);
    else
      hipLaunchKernelGGL(k_gather_rows_q<4>, dim3(qgrid), dim3(256), 0, s, V, ldv, k, Cl, ldc, n, out, ldo, row_map,
                         qe, qn, qcap, piece, vbits, newbits, pred, pred_val);
    return hipGetLastError();
  }
  const unsigned grid = (unsigned)(k < 65535 ? k : 65535);
  hipLaunchKernelGGL(k_gather_rows, dim3(grid), dim3(256), 0, s, V, ldv, k, Cl, ldc, n, init, out, ldo, row_map,
                     newbits, pred, pred_val);
  return hipGetLastError();
}
hipError_t launch_smp_round(const u64* fr, u64* fr_out, i64 ldf, u64* vis, i64 ldvis, i64 k, const i64* rp,
                            const int32_t* ci, const u64* R, i64 ldr, i64 n, u32* changed, unsigned long long* newbits,
                            const u32* pred, u32 pred_val, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  const i64 nw = words_for(n);
  if (nw > kMaxLdsWords) return hipErrorInvalidValue;
  const size_t lds = (size_t)nw * sizeof(u64);
  const unsigned grid = (unsigned)(k < 4096 ? k : 4096);
  hipLaunchKernelGGL(k_smp_round, dim3(grid), dim3(kSmpThreads), lds, s, fr, fr_out, ldf, vis, ldvis, k, rp, ci, R, ldr,
                     n, changed, newbits, pred, pred_val);
  return hipGetLastError();
}

hipError_t launch_smp_rows(const u64* V, i64 ldv, i64 k, const i64* rp, const int32_t* ci, const i64* rpt,
                           const int32_t* cit, const u64* R, i64 ldr, i64 n, int reflexive, u64* out, i64 ldo,
                           u32* iters_max, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  const i64 nw = words_for(n);
  if (3 * nw > kMaxLdsWords) return hipErrorInvalidValue;
  const size_t lds = (size_t)(3 * nw) * sizeof(u64);
  const unsigned grid = (unsigned)(k < 65535 ? k : 65535);
  if (k <= 2048)
    hipLaunchKernelGGL(k_smp_rows<8>, dim3(grid), dim3(kSmpThreads), lds, s, V, ldv, k, rp, ci, rpt, cit, R, ldr, n,
                       reflexive, out, ldo, iters_max);
  else
    hipLaunchKernelGGL(k_smp_rows<1>, dim3(grid), dim3(kSmpThreads), lds, s, V, ldv, k, rp, ci, rpt, cit, R, ldr, n,
                       reflexive, out, ldo, iters_max);
  return hipGetLastError();
}

}  // namespace bmlp
