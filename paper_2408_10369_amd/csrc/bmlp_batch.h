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
  // graphs with n >= batch_mfma_min_n() square on the matrix cores; their VALU-round items are their
  // 64-row tiles (squared there by row gathers while their 256-row block is sparse):
  u64* bt;               // R^T of the current round (n x nw), or null
  i64 mfma_rtiles;       // 256-row tiles per side (0 for the other graphs)
  i64 mfma_tile_begin;   // first matrix-core tile of this graph (mfma_rtiles^2 per round)
  i64 tblock_begin;      // first 64 x 64 transpose block of this graph (nw^2 per round)
  i64 mblock_begin;      // first 256-row block of this graph (mfma_rtiles)
};

struct BatchPlan {
  int rounds;            // kernels in the chain = largest round cap of the batch
  i64 total_rows, total_tiles, total_select_tiles;
  i64 total_qrows;       // query rows of all graphs
  bool select_by_bfs;    // answer queries by selection (BMLP-SMP) instead of reading the closure
  i64 total_mfma_tiles;  // matrix-core tiles per round, over all graphs
  i64 total_tblocks;     // transpose blocks per round, over all graphs
  i64 total_mblocks;     // 256-row blocks of the matrix-core graphs
};

// smallest n whose squarings run on the matrix cores in a batch
i64 batch_mfma_min_n();

// largest n whose queries the per-row selection kernel answers (bitmaps in registers)
i64 batch_bfs_max_n();

i64 batch_tiles(i64 n);
i64 batch_rtiles(i64 n);
i64 batch_select_tiles(i64 k, i64 n);
// words of the flag area of a batch (zeroed by the chain's setup kernel)
i64 batch_flag_words(int count, const BatchPlan& p);
// records the kernel chain on stream s (setup, rounds, select, copy); flags must hold
// batch_flag_words(count, p) words
hipError_t launch_batch_chain(BatchGraph* d_graphs, int count, const BatchPlan& p, u32* flags, hipStream_t s);

}  // namespace bmlp
