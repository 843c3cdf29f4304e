// The cost model that picks how a BMLP-RMS squaring is done (dense product, row gathers, or the
// semi-naive form), shared by the host driver and the device-side decision kernel, so that both reach
// the same choice from the same bit counts.  Not part of the public C-ABI.
#pragma once
#include "bmlp_internal.h"

namespace bmlp {

// Rates measured on MI355X at n = 16,384: dense squarings on the matrix cores (4.5e15 on a product that
// skips nothing) and on the VALU, squarings by row gathers (6.1e12 bytes/s of rows read and written over
// the density sweep's gather squarings, 7.5e12 on the largest), transposes moving the matrix in and out
// (3.2e12 bytes/s).
constexpr double kMfmaSquareOpsPerSec = 4.5e15;
constexpr double kValuSquareOpsPerSec = 1.7e15;
constexpr double kGatherBytesPerSec = 6.0e12;
constexpr double kSemiOverheadS = 50.0e-6;  // launches and the readbacks of the semi-naive route

// A squaring R.R of a sparse R is cheaper as row gathers (row i of R | R.R = R[i] | OR of the rows k over
// the set bits k of R[i], the rows read whole) than as a dense product: the gathers move about
// (bits + 3 n) rows of n bits, the dense product does 2 n^3 operations.  gather_max_n: the largest n the
// gather kernel takes.
__host__ __device__ inline bool rms_gather_pays(i64 n, i64 bits, bool mfma, i64 gather_max_n) {
  if (n > gather_max_n) return false;
  const double nn = (double)n, row_bytes = 8.0 * (double)((n + 63) >> 6);
  const double t_gather = ((double)bits + 3.0 * nn) * row_bytes / kGatherBytesPerSec;
  const double t_dense = 2.0 * nn * nn * nn / (mfma ? kMfmaSquareOpsPerSec : kValuSquareOpsPerSec);
  return t_gather < t_dense;
}

// A squaring from the bits D new in the last one: with R_t = R_{t-1} | D and R_{t-1}.R_{t-1} inside R_t,
//   R_t.R_t = R_t | R_t.D | D.R_t.
// D.R_t is a row gather over the bits of D.  R_t.D is found one of two ways:
//   columns: a column gather of R_t at the nonempty rows of D and a product with K = that number of rows;
//   transposed: (D^T . R_t^T)^T, a second row gather over the bits of D between three transposes.
// The transposed route costs about the bits of D; the column route about n^2 per nonempty row of D, so it
// only pays when D's bits crowd into few rows.  Seconds of each part:
struct SemiCost {
  double common, cols_fixed, per_row, transposed, dense;
};
__host__ __device__ inline SemiCost rms_semi_cost(i64 n, i64 dbits, bool mfma) {
  const double nn = (double)n, rb = 8.0 * (double)((n + 63) >> 6), db = (double)dbits;
  SemiCost c;
  c.common = (db + 3.0 * nn) * rb / kGatherBytesPerSec;  // D.R_t and the copy of R_t
  c.cols_fixed = 2.0 * nn * rb / 4.0e12;
  c.per_row = 2.0 * nn * nn;  // Boolean operations of the product per nonempty row of D
  c.transposed = db * rb / kGatherBytesPerSec + 3.0 * 2.0 * nn * rb / 3.2e12 + 2.0 * nn * rb / kGatherBytesPerSec;
  c.dense = 2.0 * nn * nn * nn / (mfma ? kMfmaSquareOpsPerSec : kValuSquareOpsPerSec);
  return c;
}
__host__ __device__ inline double rms_semi_cols_s(const SemiCost& c, i64 drows) {
  return c.cols_fixed + c.per_row * (double)drows / (drows >= 512 ? 3.0e15 : 1.2e15);
}
// The first test of the semi-naive route: with D's nonempty rows bounded below by ceil(dbits / n), may it
// beat the dense squaring?
__host__ __device__ inline bool rms_semi_may_pay(i64 n, i64 dbits, bool mfma) {
  if (dbits <= 0) return false;
  const SemiCost sc = rms_semi_cost(n, dbits, mfma);
  const double cols_lb = rms_semi_cols_s(sc, (dbits + n - 1) / n);
  const double alt = sc.transposed < cols_lb ? sc.transposed : cols_lb;
  return sc.common + alt + kSemiOverheadS < sc.dense;
}

// Routes of a squaring chosen on the device (k_rms_decide)
enum RmsRoute : u32 { RR_STOP = 0, RR_GATHER = 1, RR_DENSE = 2, RR_HOST = 3 };
// Per-squaring record on the device, 8 words: new bits (u64), running bit count (u64), route (u32), and a
// flag (rms_early_votes) under which the dense product's tiles vote on saturation after their first chunk
// of k, before loading ahead
constexpr int kRmsRecWords = 8;
constexpr int kRmsRecEarly = 5;

// A squaring of an R with at least a quarter of its bits set likely saturates each output tile within its
// first chunk of 512 values of k: with set bits spread at density rho, an output stays unset there with
// probability about (1 - rho^2)^512, below e^-32 from rho = 1/4.
__host__ __device__ inline bool rms_early_votes(i64 n, i64 bits) { return 4.0 * (double)bits >= (double)n * (double)n; }

}  // namespace bmlp
