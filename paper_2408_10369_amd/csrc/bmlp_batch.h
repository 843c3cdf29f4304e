// Device-side description of a batch of graphs for the batched launch.
#pragma once
#include "bmlp_internal.h"

namespace bmlp {

struct BatchGraph {
  i64 n, nw;             // nodes, data words per row
  const u64* R1; i64 ld; // input relation
  u64* closure; i64 ldc; // output R1+ (may be null)
  const u64* V; i64 k; i64 ldv;  // query rows (k may be 0)
  u64* Vstar;            // output V R1+
  u64* buf0; u64* buf1;  // ping-pong workspace, n x nw each
  i64 row_begin;         // first row of this graph in the batch-wide row numbering (max(n, k) rows each)
  i64 tile_begin;        // first product tile of this graph (tiles per round = batch_tiles(n))
  i64 rtiles;            // row tiles of the graph
  i64 smp_tile_begin;    // first selection tile of this graph
  i64 qrow_begin;        // first query row of this graph in the batch-wide query-row numbering
};

struct BatchPlan {
  int rounds;            // kernels in the chain = largest round cap of the batch
  i64 total_rows, total_tiles, total_select_tiles;
  i64 total_qrows;       // query rows of all graphs
  bool select_by_bfs;    // answer queries by selection (BMLP-SMP) instead of reading the closure
};

// largest n whose queries the per-row selection kernel answers (bitmaps in registers)
i64 batch_bfs_max_n();

i64 batch_tiles(i64 n);
i64 batch_rtiles(i64 n);
i64 batch_select_tiles(i64 k, i64 n);
// records the kernel chain on stream s (setup, rounds, select, copy); flags must hold
// count * rounds + 2 * rounds + 1 words
hipError_t launch_batch_chain(BatchGraph* d_graphs, int count, const BatchPlan& p, u32* flags, hipStream_t s);

}  // namespace bmlp
