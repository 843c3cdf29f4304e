// Batched BMLP over many graphs of uneven sizes in one hipGraph launch.
//
// For every graph g of the batch: the closure R1+ by repeated squaring
// R <- R | R.R (Section 3.3, Eq. 4 / Algorithm 1 in its R | R.R form) and the
// answers V R1+ of its query rows (Eq. 5) read off the finished closure (the
// reuse of intermediate results the paper describes in Section 4).
//
// The launch is a fixed chain of kernels captured once into a hipGraph:
//   setup        copy every R1 into the graph's ping-pong workspace, clear flags
//   round r      (r = 0 .. rounds-1) one squaring for every graph still active:
//                a persistent grid claims (graph, tile) items from an atomic
//                counter, biggest graphs first; a graph whose previous round
//                changed nothing is skipped on the device
//   select       Vstar = V . R1+ for every graph (tiles of query rows)
//   copy         the closure of every graph into its output buffer
// Round r reads buffer r & 1 and writes buffer (r + 1) & 1 of the graph, so
// the result is independent of the order in which tiles run.  Kernel
// boundaries make each round's writes visible to the next round on every XCD.
#include "bmlp_batch.h"
#include "valu_tile.h"
#include "mfma_tile.h"
#include "features.h"
#include "bmlp_mlp.h"

namespace bmlp {

namespace {

constexpr int kRPW = 16;                 // rows per wave -> 64-row tiles
constexpr int kTileRows = 4 * kRPW;
constexpr int kTileWords = 64;           // one lane per word

// the last graph whose first item of the given kind (0 VALU tile, 1 selection tile, 2 matrix-core tile,
// 3 transpose block, 4 256-row block) is at or before item t: the graph that owns t (graphs without items of that kind
// share the next graph's start and are never the last one)
__device__ __forceinline__ int find_item(const BatchGraph* __restrict__ gs, int count, i64 t, int kind) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const BatchGraph& G = gs[mid];
    const i64 b = kind == 0   ? G.tile_begin
                  : kind == 1 ? G.smp_tile_begin
                  : kind == 2 ? G.mfma_tile_begin
                  : kind == 3 ? G.tblock_begin
                              : G.mblock_begin;
    if (b <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_graph(const BatchGraph* __restrict__ gs, int count, i64 t, bool smp) {
  return find_item(gs, count, t, smp ? 1 : 0);
}

// round at which graph g stopped changing (its last product), or -1 if it
// never did within the rounds run
__device__ __forceinline__ int final_round(const u32* __restrict__ changed, int g, int rounds) {
  for (int r = 0; r < rounds; ++r)
    if (!changed[(i64)g * rounds + r]) return r;
  return -1;
}

__global__ void k_batch_setup(BatchGraph* __restrict__ gs, int count, i64 total_rows, u32* __restrict__ flags,
                              i64 nflags) {
  const i64 tid = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  const i64 nth = (i64)gridDim.x * blockDim.x;
  for (i64 i = tid; i < nflags; i += nth) flags[i] = 0u;
  // rows are numbered across graphs by row_begin, each graph's rows padded to a multiple of 8, so a group
  // of 8 rows lies in one graph: a wave takes a group (one search for its graph), lanes the words, all
  // eight rows' loads in flight
  const int lane = threadIdx.x & 63;
  const i64 wave = tid >> 6, nwaves = nth >> 6;
  for (i64 grp = wave; grp < total_rows / 8; grp += nwaves) {
    const i64 rr = grp * 8;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (gs[mid].row_begin <= rr) lo = mid; else hi = mid - 1;
    }
    const BatchGraph& G = gs[lo];
    const i64 row0 = rr - G.row_begin;
    if (row0 >= G.n) continue;
    const u64 lm = (G.n & 63) ? ((1ull << (G.n & 63)) - 1ull) : ~0ull;
    for (i64 w = lane; w < G.nw; w += 64) {
      u64 x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = row0 + r < G.n ? G.R1[(row0 + r) * G.ld + w] : 0ull;
#pragma unroll
      for (int r = 0; r < 8; ++r)
        if (row0 + r < G.n) G.buf0[(row0 + r) * G.nw + w] = w == G.nw - 1 ? x[r] & lm : x[r];
    }
  }
}

// Per graph: whether its query rows are answered by per-row selection (qsel) and whether its closure is
// computed (need), for the fixed modes; qmode 2 starts from the plain choice and k_batch_choose decides.
__global__ void k_batch_modes(const BatchGraph* __restrict__ gs, int count, int qmode, i64 bfs_words,
                              u32* __restrict__ qsel, u32* __restrict__ need) {
  const i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (g >= count) return;
  const BatchGraph& G = gs[g];
  const u32 sel = (qmode != 0 && G.k > 0 && G.nw <= bfs_words) ? 1u : 0u;
  qsel[g] = sel;
  need[g] = (G.closure_req || (G.k > 0 && !sel)) ? 1u : 0u;
}

// Statistics of each graph for the dispatcher's features: set bits of R1, its largest row count, its
// nonempty rows, and the set bits of its query rows.  Two passes and no atomics (same-address device atomics
// serialise): k_batch_stats takes a wave per group of 64 rows of a graph (max(n, k) rows, groups numbered
// batch-wide from sgroup_begin) and writes the group's four partial values; k_batch_features combines a
// graph's groups with one wave.  A group is read eight rows at a time with all their loads in flight (lanes
// over the words of a row).  The wave's graph is found by a search over the wave-uniform group index, so its
// loads are scalar.
constexpr int kStatsRows = 8;
__global__ void __launch_bounds__(256)
k_batch_stats(const BatchGraph* __restrict__ gs, int count, i64 total_groups, unsigned long long* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const i64 wave0 = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6));
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  int lo = 0;
  for (i64 grp = wave0; grp < total_groups; grp += nwaves) {
    // groups only grow along the loop, so the search starts from the last graph found
    int hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (gs[mid].sgroup_begin <= grp) lo = mid; else hi = mid - 1;
    }
    // the fields this pass reads, loaded once
    const i64 gn = gs[lo].n, gk = gs[lo].k, gnw = gs[lo].nw, gld = gs[lo].ld, gldv = gs[lo].ldv;
    const u64* __restrict__ R1 = gs[lo].R1;
    const u64* __restrict__ V = gs[lo].V;
    const u64 lm = (gn & 63) ? ((1ull << (gn & 63)) - 1ull) : ~0ull;
    const i64 rows = gn > gk ? gn : gk;
    const i64 first = (grp - gs[lo].sgroup_begin) * 64;
    const i64 last = first + 64 < rows ? first + 64 : rows;
    // a row of a graph with n < 65,536 has fewer set bits than 2^16: four rows' lane counts then share one
    // 64-bit word of 16-bit fields through the cross-lane sums (no field overflows at any partial sum)
    const bool packed = gn < 65536;
    unsigned long long bits = 0, mx = 0, nonempty = 0;  // wave-uniform after the reductions
    u32 vl = 0;                                         // this lane's set bits of the query rows
    for (i64 row0 = first; row0 < last; row0 += kStatsRows) {
      u32 pr[kStatsRows];
#pragma unroll
      for (int r = 0; r < kStatsRows; ++r) pr[r] = 0u;
      for (i64 w = lane; w < gnw; w += 64) {
        const u64 m = w == gnw - 1 ? lm : ~0ull;
        u64 xr[kStatsRows], xv[kStatsRows];
#pragma unroll
        for (int r = 0; r < kStatsRows; ++r) {
          const i64 row = row0 + r;
          xr[r] = row < last && row < gn ? R1[row * gld + w] : 0ull;
          xv[r] = row < last && row < gk ? V[row * gldv + w] : 0ull;
        }
#pragma unroll
        for (int r = 0; r < kStatsRows; ++r) {
          pr[r] += (u32)__popcll(xr[r] & m);
          vl += (u32)__popcll(xv[r] & m);
        }
      }
      u32 tot[kStatsRows];
      if (packed) {
        unsigned long long a = (unsigned long long)pr[0] | ((unsigned long long)pr[1] << 16) |
                               ((unsigned long long)pr[2] << 32) | ((unsigned long long)pr[3] << 48);
        unsigned long long b = (unsigned long long)pr[4] | ((unsigned long long)pr[5] << 16) |
                               ((unsigned long long)pr[6] << 32) | ((unsigned long long)pr[7] << 48);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          a += __shfl_xor(a, off, 64);
          b += __shfl_xor(b, off, 64);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tot[r] = (u32)((a >> (16 * r)) & 0xFFFFull);
          tot[4 + r] = (u32)((b >> (16 * r)) & 0xFFFFull);
        }
      } else {
#pragma unroll
        for (int r = 0; r < kStatsRows; ++r) {
          u32 v = pr[r];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
          tot[r] = v;
        }
      }
#pragma unroll
      for (int r = 0; r < kStatsRows; ++r) {
        bits += tot[r];
        mx = tot[r] > mx ? tot[r] : mx;
        nonempty += tot[r] ? 1u : 0u;
      }
    }
    unsigned long long vbits = vl;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vbits += __shfl_xor(vbits, off, 64);
    if (lane == 0) {
      unsigned long long* p = part + 4 * grp;
      p[0] = bits;
      p[1] = mx;
      p[2] = nonempty;
      p[3] = vbits;
    }
  }
}

// Per graph: its statistics from its groups' partial values (one wave per graph), kept in gst, and the
// dispatcher's input features.
__global__ void __launch_bounds__(256)
k_batch_features(const BatchGraph* __restrict__ gs, int count, const unsigned long long* __restrict__ part,
                 unsigned long long* __restrict__ gst, float* __restrict__ X) {
  const int lane = threadIdx.x & 63;
  const i64 g = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6));
  if (g >= count) return;
  const BatchGraph& G = gs[g];
  const i64 rows = G.n > G.k ? G.n : G.k;
  const i64 groups = (rows + 63) / 64;
  unsigned long long b = 0, mx = 0, ne = 0, vb = 0;
  for (i64 i = lane; i < groups; i += 64) {
    const unsigned long long* p = part + 4 * (G.sgroup_begin + i);
    b += p[0];
    mx = p[1] > mx ? p[1] : mx;
    ne += p[2];
    vb += p[3];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    b += __shfl_xor(b, off, 64);
    const unsigned long long m2 = __shfl_xor(mx, off, 64);
    mx = m2 > mx ? m2 : mx;
    ne += __shfl_xor(ne, off, 64);
    vb += __shfl_xor(vb, off, 64);
  }
  if (lane == 0) {
    unsigned long long* s = gst + 4 * g;
    s[0] = b;
    s[1] = mx;
    s[2] = ne;
    s[3] = vb;
    make_features(X + kIn * g, (double)G.n, (double)b, (double)mx, (double)ne, (double)G.k,
                  G.closure_req ? 0.5f : 0.f, 1, 0, (double)vb, (double)vb, 0.0, 0);
  }
}

// The model's choice per graph between reading its answers off the closure (output 2) and per-row
// selection (output 3, the one-launch selection's prediction), where the selection kernel takes the graph.
__global__ void k_batch_choose(const BatchGraph* __restrict__ gs, int count, i64 bfs_words, const float* __restrict__ Y,
                               u32* __restrict__ qsel, u32* __restrict__ need) {
  const i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (g >= count) return;
  const BatchGraph& G = gs[g];
  // a closure that is an output is computed anyway, and reading the answers off it (the closure rows of
  // each query row's sources) costs less than expanding them by selection: the model is asked only where
  // the closure would be computed for the queries alone
  const bool can_select = G.k > 0 && G.nw <= bfs_words && !G.closure_req;
  const u32 sel = (can_select && Y[kOut * g + 3] < Y[kOut * g + 2]) ? 1u : 0u;  // ties keep the closure
  qsel[g] = sel;
  need[g] = (G.closure_req || (G.k > 0 && !sel)) ? 1u : 0u;
}

// Rows row0 .. row0 + kRPW - 1 of R | R.R by row gathers (row i = R[i] | OR of the rows k over the
// set bits k of R[i]), one wave, lane l owning word l (nw <= 64).  The set bits of a row are walked in
// batches of eight (across its words), so that eight row loads are in flight at a time.
__device__ __forceinline__ int gather_square_rows(const u64* __restrict__ cur, u64* __restrict__ nxt, i64 n, i64 nw,
                                                  i64 row0, int lane) {
  int ch = 0;
  for (int r = 0; r < kRPW; ++r) {
    const i64 row = row0 + r;
    if (row >= n) break;
    const u64 mine = lane < nw ? cur[row * nw + lane] : 0ull;
    u64 acc = mine;
    u64 nzw = __ballot(mine != 0ull);  // words of the row with set bits (wave-uniform)
    // the walk over the row's set bits is wave-uniform and kept in scalar registers
    int w = 0;
    u64 x = 0ull;
    const int lc = lane < nw ? lane : (int)nw - 1;
    for (;;) {
      int src[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (!x && nzw) {
          w = __ffsll((unsigned long long)nzw) - 1;
          nzw &= nzw - 1;
          x = uniform64(__shfl(mine, w, 64));
        }
        src[q] = -1;
        if (x) {
          src[q] = 64 * w + (__ffsll((unsigned long long)x) - 1);
          x &= x - 1;
        }
      }
      if (src[0] < 0) break;
      // unguarded loads, all eight in flight: a missing source repeats src[0] and is masked out
      u64 t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = cur[(i64)(src[q] >= 0 ? src[q] : src[0]) * nw + lc];
      u64 v = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) v |= src[q] >= 0 ? t[q] : 0ull;
      acc |= v;
    }
    if (lane < nw) {
      nxt[row * nw + lane] = acc;
      ch |= acc != mine;
    }
  }
  return ch;
}

// Sparse or dense, per 256-row block of the graphs that square on the matrix cores, for this round: a
// block with fewer than n set bits (density under 1/256) is squared by row gathers, a denser one on the
// matrix cores (whose graph then needs R^T).  The gathers of a wave walk a row's bits in batches of
// eight loads, so they are latency-bound and pay only well below the density where a VALU tile would
// break even (measured on the 512-graph batch: thresholds n / 4, n and 4 n gave 17.9, 16.6 and
// 21.2 ms).  One workgroup per block.
__global__ void __launch_bounds__(256)
k_batch_decide(const BatchGraph* __restrict__ gs, int count, i64 total_blocks, int round, int rounds,
               const u32* __restrict__ changed, const u32* __restrict__ any_active, u32* __restrict__ bdense,
               u32* __restrict__ gdense, const u32* __restrict__ need) {
  __shared__ u32 bits_w[4];
  if (round > 0 && any_active[round - 1] == 0u) return;  // every graph has converged
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (i64 b = blockIdx.x; b < total_blocks; b += gridDim.x) {
    const int g = find_item(gs, count, b, 4);
    if (!need[g] || (round > 0 && !changed[(i64)g * rounds + round - 1])) continue;
    const BatchGraph& G = gs[g];
    const i64 blk = b - G.mblock_begin;
    const u64* cur = (round & 1) ? G.buf1 : G.buf0;
    u32 pc = 0;
    for (i64 e = threadIdx.x; e < 256 * G.nw; e += 256) {
      const i64 row = blk * 256 + e / G.nw;
      if (row < G.n) pc += (u32)__popcll(cur[row * G.nw + e % G.nw]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off, 64);
    if (lane == 0) bits_w[wave] = pc;
    __syncthreads();
    if (threadIdx.x == 0) {
      const i64 bits = (i64)bits_w[0] + bits_w[1] + bits_w[2] + bits_w[3];
      const u32 dense = (bits >= G.n || G.nw > 64) ? 1u : 0u;
      bdense[b] = dense;
      if (dense) atomicOr(&gdense[(i64)g * rounds + round], 1u);
    }
    __syncthreads();
  }
}

// Items taken per atomic on a work queue's counter.  Tiles of one graph are numbered together and the big
// graphs come first, so taking several at a time gives one workgroup a run of expensive tiles: four per
// fetch made the 512-graph batch 16% slower than one.
constexpr int kFetch = 1;

__global__ void __launch_bounds__(256)
k_batch_round(const BatchGraph* __restrict__ gs, int count, i64 total_tiles, int round, int rounds,
              u32* __restrict__ changed, u32* __restrict__ counters, u32* __restrict__ any_active,
              const u32* __restrict__ bdense, const u32* __restrict__ need) {
  __shared__ u64 Bs[64][kTileWords];
  __shared__ i64 item;
  __shared__ u32 tile_bits[4];
  __shared__ u32 tile_ch[4];  // per wave: the last tile changed one of its rows
  if (round > 0 && any_active[round - 1] == 0u) return;  // every graph has converged
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x < 4) tile_ch[threadIdx.x] = 0u;
  // thread 0: the items of the current fetch, the graph of the last tile, and the flags this workgroup has
  // set this round (tiles come in increasing order, so a graph's tiles are contiguous for a workgroup):
  // each flag is written once per workgroup rather than once per wave and tile
  i64 next = 0, end = 0;
  int prev_g = -1, set_g = -1;
  bool set_any = false;
  for (;;) {
    if (threadIdx.x == 0) {
      if (next == end) {
        next = (i64)atomicAdd(&counters[round], (u32)kFetch);
        end = next + kFetch;
      }
      item = next++;
    }
    __syncthreads();
    const i64 t = item;
    if (threadIdx.x == 0) {
      const u32 c = tile_ch[0] | tile_ch[1] | tile_ch[2] | tile_ch[3];
      tile_ch[0] = tile_ch[1] = tile_ch[2] = tile_ch[3] = 0u;
      if (c && prev_g >= 0) {
        if (prev_g != set_g) {
          atomicOr(&changed[(i64)prev_g * rounds + round], 1u);
          set_g = prev_g;
        }
        if (!set_any) {
          atomicOr(&any_active[round], 1u);
          set_any = true;
        }
      }
    }
    __syncthreads();
    if (t >= total_tiles) break;
    const int g = find_graph(gs, count, t, false);
    if (threadIdx.x == 0) prev_g = g;
    if (!need[g] || (round > 0 && !changed[(i64)g * rounds + round - 1])) continue;
    const BatchGraph& G = gs[g];
    const i64 local = t - G.tile_begin;
    const u64* cur = (round & 1) ? G.buf1 : G.buf0;
    u64* nxt = (round & 1) ? G.buf0 : G.buf1;
    if (G.mfma_rtiles) {
      // 64-row tile `local` of a graph that squares on the matrix cores: squared here by row gathers while
      // its 256-row block is sparse, by k_batch_round_mfma once it is dense
      if (bdense[G.mblock_begin + (local >> 2)]) continue;
      const int ch = gather_square_rows(cur, nxt, G.n, G.nw, local * kTileRows + (i64)wave * kRPW, lane);
      const u64 bch = __ballot(ch);
      if (lane == 0) tile_ch[wave] = bch != 0ull ? 1u : 0u;
      continue;
    }
    const i64 rt = local % G.rtiles, ct = local / G.rtiles;
    const i64 row0 = rt * kTileRows + (i64)wave * kRPW;
    const i64 w0 = ct * kTileWords;
    // A tile of a still sparse R (fewer set bits than n in its 64 rows, i.e. density under 1/64) is
    // squared by row gathers; the dense tile product costs the same whatever the density.
    bool gather = false;
    if (G.nw <= kTileWords) {
      u32 pc = 0;
      const i64 lc = lane < G.nw ? lane : G.nw - 1;
      u64 t[kRPW];
#pragma unroll
      for (int r = 0; r < kRPW; ++r) t[r] = cur[(row0 + r < G.n ? row0 + r : G.n - 1) * G.nw + lc];
#pragma unroll
      for (int r = 0; r < kRPW; ++r)
        if (row0 + r < G.n && lane < G.nw) pc += (u32)__popcll(t[r]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off, 64);
      if (lane == 0) tile_bits[wave] = pc;
      __syncthreads();
      gather = (i64)tile_bits[0] + tile_bits[1] + tile_bits[2] + tile_bits[3] < G.n;
      __syncthreads();
    }
    int ch;
    if (gather) {
      ch = gather_square_rows(cur, nxt, G.n, G.nw, row0, lane);
    } else {
      u32 acc[kRPW][1][2];
#pragma unroll
      for (int r = 0; r < kRPW; ++r) acc[r][0][0] = acc[r][0][1] = 0u;
      valu_tile_accumulate<kRPW, 1>(cur, G.nw, cur, G.nw, G.n, G.n, G.nw, row0, w0, 0, G.nw, Bs, acc);
      ch = valu_tile_store<kRPW, 1>(acc, cur, G.nw, nxt, G.nw, nullptr, 0, G.n, G.nw, row0, w0);
    }
    const u64 bch = __ballot(ch);
    if (lane == 0) tile_ch[wave] = bch != 0ull ? 1u : 0u;
  }
}

// R^T of the current round for the graphs that square on the matrix cores (the product consumes B^T):
// one wave per 64 x 64 bit block, 64 ballots.
__global__ void __launch_bounds__(256)
k_batch_transpose(const BatchGraph* __restrict__ gs, int count, i64 total_blocks, int round, int rounds,
                  const u32* __restrict__ changed, const u32* __restrict__ any_active,
                  const u32* __restrict__ gdense, const u32* __restrict__ need) {
  if (round > 0 && any_active[round - 1] == 0u) return;  // every graph has converged
  const int lane = threadIdx.x & 63;
  const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6;
  const i64 nwaves = ((i64)gridDim.x * blockDim.x) >> 6;
  for (i64 bi = wave; bi < total_blocks; bi += nwaves) {
    const int g = find_item(gs, count, bi, 3);
    if (!need[g] || (round > 0 && !changed[(i64)g * rounds + round - 1])) continue;
    if (!gdense[(i64)g * rounds + round]) continue;  // every block of the graph is squared by gathers
    const BatchGraph& G = gs[g];
    const i64 local = bi - G.tblock_begin;
    const i64 rb = local / G.nw, cw = local - rb * G.nw;  // rows 64 rb .., word cw of R
    const u64* cur = (round & 1) ? G.buf1 : G.buf0;
    const i64 r = rb * 64 + lane;
    const u64 x = r < G.n ? cur[r * G.nw + cw] : 0ull;
    u64 mine = 0;
#pragma unroll 8
    for (int j = 0; j < 64; ++j) {
      const u64 b = __ballot((x >> j) & 1ull);
      if (lane == j) mine = b;
    }
    const i64 orow = cw * 64 + lane;  // row of R^T = column of R
    if (orow < G.n) G.bt[orow * G.nw + rb] = mine;
  }
}

// One round for the graphs that square on the matrix cores: one 8-wave workgroup per (graph, 256 x 256
// tile), a matrix-core product of R by R^T; the tiles of a block k_batch_decide found sparse are left
// to the row gathers of k_batch_round.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_batch_round_mfma(const BatchGraph* __restrict__ gs, int count, int round, int rounds, u32* __restrict__ changed,
                   u32* __restrict__ any_active, const u32* __restrict__ bdense, const u32* __restrict__ need) {
  __shared__ MfmaLds L;
  if (round > 0 && any_active[round - 1] == 0u) return;  // every graph has converged
  const i64 t = blockIdx.x;  // one workgroup per tile; tiles are numbered biggest graphs first
  const int g = find_item(gs, count, t, 2);
  if (!need[g] || (round > 0 && !changed[(i64)g * rounds + round - 1])) return;
  const BatchGraph& G = gs[g];
  const i64 local = t - G.mfma_tile_begin;
  const i64 tr = local / G.mfma_rtiles, tc = local - tr * G.mfma_rtiles;
  const u64* cur = (round & 1) ? G.buf1 : G.buf0;
  u64* nxt = (round & 1) ? G.buf0 : G.buf1;
  if (!bdense[G.mblock_begin + tr]) return;  // a still sparse block: squared by k_batch_round
  const MfmaTile mt{cur, G.nw, G.bt, G.nw, cur, G.nw, nxt, G.nw, nullptr, 0, G.n, G.n, G.n,
                    &changed[(i64)g * rounds + round], nullptr, nullptr, &any_active[round]};
  mfma_tile(L, mt, tr, tc);
}

__global__ void __launch_bounds__(256)
k_batch_select(const BatchGraph* __restrict__ gs, int count, i64 total_tiles, int rounds,
               const u32* __restrict__ changed, u32* __restrict__ counter, const u32* __restrict__ qsel) {
  __shared__ u64 Bs[64][kTileWords];
  __shared__ i64 item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  i64 next = 0, end = 0;  // thread 0: the items of the current fetch
  for (;;) {
    if (threadIdx.x == 0) {
      if (next == end) {
        next = (i64)atomicAdd(counter, (u32)kFetch);
        end = next + kFetch;
      }
      item = next++;
    }
    __syncthreads();
    const i64 t = item;
    __syncthreads();
    if (t >= total_tiles) break;
    const int g = find_graph(gs, count, t, true);
    const BatchGraph& G = gs[g];
    if (qsel[g]) continue;  // answered by the selection kernel
    const int fr = final_round(changed, g, rounds);
    const u64* clo = ((fr + 1) & 1) ? G.buf1 : G.buf0;  // buffer written by the last round
    const i64 local = t - G.smp_tile_begin;
    const i64 vrt = (G.k + kTileRows - 1) / kTileRows;
    const i64 rt = local % vrt, ct = local / vrt;
    const i64 row0 = rt * kTileRows + (i64)wave * kRPW;
    const i64 w0 = ct * kTileWords;
    u32 acc[kRPW][1][2];
#pragma unroll
    for (int r = 0; r < kRPW; ++r) acc[r][0][0] = acc[r][0][1] = 0u;
    valu_tile_accumulate<kRPW, 1>(G.V, G.ldv, clo, G.nw, G.k, G.n, G.nw, row0, w0, 0, G.nw, Bs, acc);
    (void)valu_tile_store<kRPW, 1>(acc, nullptr, 0, G.Vstar, G.ldv, nullptr, 0, G.k, G.nw, row0, w0);
  }
}

// Selection without the closure for the graphs of n <= 64 kMsWords: the semi-naive fixpoint of Eq. 5 for 64
// query rows at once, transposed.  One workgroup per graph keeps, per node u, the 64-bit masks vis[u]
// (which of the chunk's query rows have reached u) and fr[u] (rows that reached u and are not yet pushed
// along u's edges) in LDS.  A wave takes the nodes of a 64-node block whose fr is nonzero, clears it, loads
// their bit rows of R1 (eight rows in flight) and pushes the mask along every edge u -> v:
//   old = vis[v] |= f; fr[v] |= f & ~old
// so each (query row, node) pair enters fr once per time it enters vis, and the fixpoint is the
// selection's: vis = V_chunk R1+ (transposed), in whatever order the pushes happen.  A pass over all nodes
// that finds no nonzero fr ends the fixpoint.  One 512-byte row load serves 64 query rows, where the
// per-row kernel below loads it once per row.
constexpr int kMsWords = 64;  // n <= 4,096
constexpr int kMsThreads = 512;

__global__ void __launch_bounds__(kMsThreads)
k_batch_select_ms(const BatchGraph* __restrict__ gs, int count, i64 nmax, const u32* __restrict__ qsel) {
  extern __shared__ u64 msh[];
  u64* fr = msh;
  u64* vis = msh + nmax;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int kWaves = kMsThreads / 64;
  for (i64 g = blockIdx.x; g < count; g += gridDim.x) {
    const BatchGraph& G = gs[g];
    if (!qsel[g] || G.k == 0 || G.n == 0 || G.nw > kMsWords || G.n > nmax) continue;  // uniform per workgroup
    const i64 n = G.n, nw = G.nw;
    const u64 lm = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
    for (i64 c0 = 0; c0 < G.k; c0 += 64) {
      const int kc = (int)(G.k - c0 < 64 ? G.k - c0 : 64);
      // fr[u] = the query rows of the chunk with bit u set (a 64 x 64 bit transpose per node block)
      for (i64 i = wave; i < nw; i += kWaves) {
        u64 x = lane < kc ? G.V[(c0 + lane) * G.ldv + i] : 0ull;
        if (i == nw - 1) x &= lm;
        u64 mine = 0ull;
        for (int b = 0; b < 64; ++b) {
          const u64 bal = __ballot((x >> b) & 1ull);
          if (lane == b) mine = bal;
        }
        if (64 * i + lane < n) {
          fr[64 * i + lane] = mine;
          vis[64 * i + lane] = 0ull;
        }
      }
      __syncthreads();
      for (;;) {
        int did = 0;
        for (i64 i = wave; i < nw; i += kWaves) {
          const i64 u = 64 * i + lane;
          const u64 f = u < n ? atomicExch((unsigned long long*)&fr[u], 0ull) : 0ull;
          u64 m = __ballot(f != 0ull);
          did |= m != 0ull;
          while (m) {
            int ln[8];
            int cnt = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
              ln[c] = 0;
              if (m) {
                ln[c] = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                ++cnt;
              }
            }
            u64 row[8];
#pragma unroll
            for (int c = 0; c < 8; ++c)
              row[c] = (c < cnt && lane < nw) ? G.R1[(64 * i + ln[c]) * G.ld + lane] & (lane == nw - 1 ? lm : ~0ull)
                                              : 0ull;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
              if (c >= cnt) break;
              const u64 fu = __shfl(f, ln[c], 64);
              u64 x = row[c];
              while (x) {
                const int b = __ffsll((unsigned long long)x) - 1;
                x &= x - 1;
                const i64 v = 64 * (i64)lane + b;
                const u64 old = atomicOr((unsigned long long*)&vis[v], fu);
                const u64 nb = fu & ~old;
                if (nb) atomicOr((unsigned long long*)&fr[v], nb);
              }
            }
          }
        }
        if (!__syncthreads_or(did)) break;
      }
      // answer rows c0 .. c0 + kc - 1, word i: the transpose of vis over node block i
      for (i64 i = wave; i < nw; i += kWaves) {
        const u64 v = 64 * i + lane < n ? vis[64 * i + lane] : 0ull;
        u64 mine = 0ull;
        for (int q = 0; q < kc; ++q) {
          const u64 bal = __ballot((v >> q) & 1ull);
          if (lane == q) mine = bal;
        }
        if (lane < kc) G.Vstar[(c0 + lane) * G.ldv + i] = mine;
      }
      __syncthreads();
    }
  }
}

// Selection without the closure (the plain schedule's reading of a partially grounded query as
// BMLP-SMP): one wave per query row runs the semi-naive fixpoint of Eq. 5 with its frontier,
// visited and successor bitmaps in registers (lane l owns words l, l + 64, ...; up to kBfsWords
// words), expanding a frontier node u by OR-ing its bit row R1[u, :].  The set bits of the
// frontier are walked uniformly across the wave (ballot of nonzero words, then the bits of each).
constexpr int kBfsWords = 256;  // n <= 16,384
constexpr int kBfsPer = kBfsWords / 64;

__global__ void __launch_bounds__(256)
k_batch_select_bfs(const BatchGraph* __restrict__ gs, int count, i64 total_qrows, u32* __restrict__ counter,
                   const u32* __restrict__ qsel) {
  __shared__ i64 item[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (;;) {
    if (lane == 0) item[wv] = (i64)atomicAdd(counter, 1u);
    __builtin_amdgcn_wave_barrier();
    const i64 it = item[wv];
    __builtin_amdgcn_wave_barrier();
    if (it >= total_qrows) break;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (gs[mid].qrow_begin <= it) lo = mid; else hi = mid - 1;
    }
    const BatchGraph& G = gs[lo];
    const i64 row = it - G.qrow_begin;
    // answered off the closure, or by the multi-row kernel above
    if (row >= G.k || G.nw > kBfsWords || G.nw <= kMsWords || !qsel[lo]) continue;
    const u64 lm = (G.n & 63) ? ((1ull << (G.n & 63)) - 1ull) : ~0ull;
    u64 fr[kBfsPer], vis[kBfsPer], nxt[kBfsPer];
#pragma unroll
    for (int j = 0; j < kBfsPer; ++j) {
      const i64 w = lane + 64 * j;
      fr[j] = (w < G.nw) ? (G.V[row * G.ldv + w] & (w == G.nw - 1 ? lm : ~0ull)) : 0ull;
      vis[j] = 0ull;
    }
    for (i64 round = 0; round <= G.n + 1; ++round) {
#pragma unroll
      for (int j = 0; j < kBfsPer; ++j) nxt[j] = 0ull;
#pragma unroll
      for (int j = 0; j < kBfsPer; ++j) {
        u64 lanes = __ballot(fr[j] != 0ull);
        while (lanes) {
          const int src = __ffsll((unsigned long long)lanes) - 1;
          lanes &= lanes - 1;
          u64 x = __shfl(fr[j], src, 64);
          while (x) {
            const int b = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            const i64 u = (i64)(src + 64 * j) * 64 + b;
#pragma unroll
            for (int q = 0; q < kBfsPer; ++q) {
              const i64 w = lane + 64 * q;
              if (w < G.nw) nxt[q] |= G.R1[u * G.ld + w];
            }
          }
        }
      }
      int any = 0;
#pragma unroll
      for (int j = 0; j < kBfsPer; ++j) {
        const i64 w = lane + 64 * j;
        const u64 nv = nxt[j] & ~vis[j] & (w == G.nw - 1 ? lm : ~0ull);
        vis[j] |= nv;
        fr[j] = nv;
        any |= nv != 0ull;
      }
      if (__ballot(any) == 0ull) break;
    }
#pragma unroll
    for (int j = 0; j < kBfsPer; ++j) {
      const i64 w = lane + 64 * j;
      if (w < G.nw) G.Vstar[row * G.ldv + w] = vis[j];
    }
  }
}

// closure rows into the outputs (with the caller's leading dimension, padding words zeroed) and the
// padding words of the answer rows
__global__ void k_batch_copy(const BatchGraph* __restrict__ gs, int count, i64 total_rows, int rounds,
                             const u32* __restrict__ changed) {
  const i64 tid = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  const i64 nth = (i64)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const i64 wave = tid >> 6, nwaves = nth >> 6;
  // groups of 8 rows of one graph, as in k_batch_setup
  for (i64 grp = wave; grp < total_rows / 8; grp += nwaves) {
    const i64 rr = grp * 8;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (gs[mid].row_begin <= rr) lo = mid; else hi = mid - 1;
    }
    const BatchGraph& G = gs[lo];
    const i64 row0 = rr - G.row_begin;
    if (G.closure && row0 < G.n) {
      const int fr = final_round(changed, lo, rounds);
      const u64* clo = ((fr + 1) & 1) ? G.buf1 : G.buf0;
      for (i64 w = lane; w < G.ldc; w += 64) {
        u64 x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = (row0 + r < G.n && w < G.nw) ? clo[(row0 + r) * G.nw + w] : 0ull;
#pragma unroll
        for (int r = 0; r < 8; ++r)
          if (row0 + r < G.n) G.closure[(row0 + r) * G.ldc + w] = x[r];
      }
    }
    for (int r = 0; r < 8; ++r)
      if (row0 + r < G.k)
        for (i64 w = G.nw + lane; w < G.ldv; w += 64) G.Vstar[(row0 + r) * G.ldv + w] = 0ull;
  }
}

int grid_cap(i64 work, int cap) {
  if (work < 1) return 1;
  return (int)(work < cap ? work : cap);
}

}  // namespace

i64 batch_tiles(i64 n) {
  const i64 nw = words_for(n);
  return ((n + kTileRows - 1) / kTileRows) * ((nw + kTileWords - 1) / kTileWords);
}

i64 batch_rtiles(i64 n) { return (n + kTileRows - 1) / kTileRows; }

i64 batch_bfs_max_n() { return (i64)kBfsWords * 64; }

i64 batch_ms_max_n() { return (i64)kMsWords * 64; }

// A graph of at least one whole 256 x 256 tile squares its dense blocks on the matrix cores: on the
// 512-graph batch (n from 64 to 4,096) the threshold at 256 ran 12.5 ms, at 512 12.8 ms, at 1,024 13.7 ms,
// at 2,048 15.9 ms (plain schedule).
i64 batch_mfma_min_n() { return 256; }

i64 batch_qsel_offset(int count, const BatchPlan& p) {
  const i64 w = 2 * (i64)count * p.rounds + 2 * (i64)p.rounds + 2 + p.total_mblocks;
  return (w + 1) & ~(i64)1;  // 8-byte aligned for the statistics that follow
}

// per graph after qsel: need (1), statistics (4 u64), features (16 float), model outputs (4 float); then
// (aligned) the statistics pass's partial values, 4 u64 per 64-row group
i64 batch_flag_words(int count, const BatchPlan& p) {
  return batch_qsel_offset(count, p) + (i64)count * (1 + 1 + 8 + kIn + kOut) + 2 + 8 * p.total_sgroups + 2;
}

i64 batch_select_tiles(i64 k, i64 n) {
  const i64 nw = words_for(n);
  return ((k + kTileRows - 1) / kTileRows) * ((nw + kTileWords - 1) / kTileWords);
}

hipError_t launch_batch_chain(BatchGraph* d_graphs, int count, const BatchPlan& p, u32* flags, const float* model,
                              hipStream_t s) {
  // flags layout: changed[count * rounds] | any_active[rounds] | counters[rounds + 2] |
  //               gdense[count * rounds] | bdense[total_mblocks] | (aligned) qsel[count] | need[count] |
  //               (aligned) stats[count][4 u64] | X[count][16] | Y[count][4] | (aligned) part[total_sgroups][4 u64]
  u32* changed = flags;
  u32* any_active = flags + (i64)count * p.rounds;
  u32* counters = any_active + p.rounds;
  u32* gdense = counters + p.rounds + 2;
  u32* bdense = gdense + (i64)count * p.rounds;
  u32* qsel = flags + batch_qsel_offset(count, p);
  u32* need = qsel + count;
  unsigned long long* gst = (unsigned long long*)(flags + ((batch_qsel_offset(count, p) + 2 * (i64)count + 1) & ~(i64)1));
  float* X = (float*)(gst + 4 * (i64)count);
  float* Y = X + (i64)kIn * count;
  unsigned long long* part =
      (unsigned long long*)(flags + ((((u32*)(Y + (i64)kOut * count)) - flags + 1) & ~(i64)1));
  const i64 nflags = batch_flag_words(count, p);
  hipLaunchKernelGGL(k_batch_setup, dim3(grid_cap((p.total_rows / 8 * 64 + 255) / 256, 8192)), dim3(256), 0, s, d_graphs,
                     count, p.total_rows, flags, nflags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned ggrid = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(k_batch_modes, dim3(ggrid), dim3(256), 0, s, (const BatchGraph*)d_graphs, count, p.qmode,
                     (i64)kBfsWords, qsel, need);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (p.qmode == 2 && model) {
    // the dispatcher's choice per graph, on the device: statistics, features, the network, the argmin
    hipLaunchKernelGGL(k_batch_stats, dim3(grid_cap((p.total_sgroups * 64 + 255) / 256, 8192)), dim3(256), 0, s,
                       (const BatchGraph*)d_graphs, count, p.total_sgroups, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_features, dim3((unsigned)((count * 64ll + 255) / 256)), dim3(256), 0, s,
                       (const BatchGraph*)d_graphs, count, (const unsigned long long*)part, gst, X);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_mlp_forward(model, model + kParams, model + kParams + kIn, X, count, nullptr, nullptr, Y, s)) !=
        hipSuccess)
      return e;
    hipLaunchKernelGGL(k_batch_choose, dim3(ggrid), dim3(256), 0, s, (const BatchGraph*)d_graphs, count,
                       (i64)kBfsWords, (const float*)Y, qsel, need);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int pgrid = grid_cap(p.total_tiles, 1024);
  for (int r = 0; r < p.rounds; ++r) {
    if (p.total_mblocks > 0) {
      hipLaunchKernelGGL(k_batch_decide, dim3(grid_cap(p.total_mblocks, 4096)), dim3(256), 0, s,
                         (const BatchGraph*)d_graphs, count, p.total_mblocks, r, p.rounds, (const u32*)changed,
                         (const u32*)any_active, bdense, gdense, (const u32*)need);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (p.total_tiles > 0) {
      hipLaunchKernelGGL(k_batch_round, dim3(pgrid), dim3(256), 0, s, (const BatchGraph*)d_graphs, count,
                         p.total_tiles, r, p.rounds, changed, counters, any_active, (const u32*)bdense,
                         (const u32*)need);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (p.total_mfma_tiles > 0) {
      hipLaunchKernelGGL(k_batch_transpose, dim3(grid_cap((p.total_tblocks * 64 + 255) / 256, 8192)), dim3(256), 0, s,
                         (const BatchGraph*)d_graphs, count, p.total_tblocks, r, p.rounds, (const u32*)changed,
                         (const u32*)any_active, (const u32*)gdense, (const u32*)need);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_batch_round_mfma, dim3((unsigned)p.total_mfma_tiles), dim3(512), 0, s,
                         (const BatchGraph*)d_graphs, count, r, p.rounds, changed, any_active, (const u32*)bdense,
                         (const u32*)need);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (p.qmode != 0 && p.ms_max_n > 0) {
    hipLaunchKernelGGL(k_batch_select_ms, dim3((unsigned)count), dim3(kMsThreads),
                       (size_t)(2 * p.ms_max_n) * sizeof(u64), s, (const BatchGraph*)d_graphs, count, p.ms_max_n,
                       (const u32*)qsel);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.qmode != 0 && p.total_qrows > p.ms_qrows) {
    hipLaunchKernelGGL(k_batch_select_bfs, dim3(grid_cap((p.total_qrows + 3) / 4, 2048)), dim3(256), 0, s,
                       (const BatchGraph*)d_graphs, count, p.total_qrows, counters + p.rounds + 1, (const u32*)qsel);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.total_select_tiles > 0) {
    hipLaunchKernelGGL(k_batch_select, dim3(grid_cap(p.total_select_tiles, 1024)), dim3(256), 0, s,
                       (const BatchGraph*)d_graphs, count, p.total_select_tiles, p.rounds, (const u32*)changed,
                       counters + p.rounds, (const u32*)qsel);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_batch_copy, dim3(grid_cap((p.total_rows / 8 * 64 + 255) / 256, 8192)), dim3(256), 0, s,
                     (const BatchGraph*)d_graphs, count, p.total_rows, p.rounds, (const u32*)changed);
  return hipGetLastError();
}

}  // namespace bmlp
