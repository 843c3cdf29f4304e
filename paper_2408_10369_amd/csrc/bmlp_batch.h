// Device-side description of a batch of graphs for the batched launch.
#pragma once
#include "bmlp_internal.h"

namespace bmlp {

struct BatchGraph {
  i64 n, nw;             // nodes, data words per row
  i64 closure_req;       // the caller asked for the closure (it is an output)
  const u64* R1; i64 ld; // input relation
  u64* closure; i64 ldc; // output R1+ (may be null)
  const u64* V; i64 k; i64 ldv;  // query rows (k may be 0)
  u64* Vstar;            // output V R1+
  u64* buf0; u64* buf1;  // ping-pong workspace, n x nw each
  i64 row_begin;         // first row of this graph in the batch-wide row numbering (max(n, k) rows each,
                         // rounded up to a multiple of 8)
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
  i64 sgroup_begin;      // first 64-row group of this graph's statistics pass (max(n, k) rows)
};

struct BatchPlan {
  int rounds;            // kernels in the chain = largest round cap of the batch
  i64 total_rows, total_tiles, total_select_tiles;
  i64 total_qrows;       // query rows of all graphs
  int qmode;             // how query rows are answered: 0 off the closures; 1 by per-row selection (BMLP-SMP)
                         // where the selection kernel takes the graph (the paper's mapping); 2 per graph
                         // as the dispatcher model chooses on the device (qsel below)
  i64 total_mfma_tiles;  // matrix-core tiles per round, over all graphs
  i64 total_tblocks;     // transpose blocks per round, over all graphs
  i64 total_mblocks;     // 256-row blocks of the matrix-core graphs
  i64 ms_max_n;          // largest n of the graphs with query rows whose selection runs 64 rows at a time
                         // (n <= batch_ms_max_n(); 0: none)
  i64 ms_qrows;          // query rows of those graphs
  i64 total_sgroups;     // 64-row groups of the statistics pass, over all graphs
};

// largest n whose query rows the batch selects 64 at a time (masks per node in LDS)
i64 batch_ms_max_n();

// smallest n whose squarings run on the matrix cores in a batch
i64 batch_mfma_min_n();

// largest n whose queries the per-row selection kernel answers (bitmaps in registers)
i64 batch_bfs_max_n();

i64 batch_tiles(i64 n);
i64 batch_rtiles(i64 n);
i64 batch_select_tiles(i64 k, i64 n);
// words of the flag area of a batch (zeroed by the chain's setup kernel)
i64 batch_flag_words(int count, const BatchPlan& p);
// records the kernel chain on stream s (setup, the per-graph modes, rounds, select, copy); flags must hold
// batch_flag_words(count, p) words.  model: the dispatcher's parameters | mu | sd on the device (qmode 2).
// Per graph the flag area ends with: qsel (1 = its query rows are answered by per-row selection), need
// (1 = its closure is computed), and for qmode 2 its statistics, features and the model's outputs.
hipError_t launch_batch_chain(BatchGraph* d_graphs, int count, const BatchPlan& p, u32* flags, const float* model,
                              hipStream_t s);
// offsets (words) of the per-graph areas in the flag area
i64 batch_qsel_offset(int count, const BatchPlan& p);

}  // namespace bmlp
