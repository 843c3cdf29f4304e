/*
 * bmlp.h -- C ABI of libbmlp: Boolean Matrix Logic Programming (Ai,
 * "Boolean Matrix Logic Programming on the GPU", arXiv 2408.10369) on AMD
 * Instinct MI355X (gfx950).
 *
 * The library evaluates linear dyadic recursive datalog bottom-up by
 * Boolean-semiring (OR, AND) matrix products:
 *   bmlp_rms             BMLP-RMS, repeated squaring to the closure R1+
 *                        (Section 3.3, Eqs. 2-4; Algorithm 1)
 *   bmlp_smp             BMLP-SMP, selective products v R1+ from chosen
 *                        source rows (Section 3.3, Eq. 5; Algorithm 2)
 *   bmlp_compose_linear  general linear recursion p <- b; p <- s, p, i.e.
 *                        P = Rs* Rb (Section 3.4, Theorem 1)
 *   bmlp_compose_two_sided  p <- b; p <- l, p, r (e.g. same-generation)
 *   bmlp_closure_insert  a closure kept up to date under edge insertions
 *                        (dynamic databases, the conclusion's future work)
 * plus the Boolean matrix operators they are built from (Section 2 and
 * Section 4: addition, multiplication, transpose, negation) and the packing
 * of facts into matrices (Section 3.2).
 *
 * ---------------------------------------------------------------- layout
 * A relation r over constants c_0..c_{n-1} (indices from the bijection of
 * Section 3.2) is an n x n Boolean matrix with R_ij = 1 iff r(c_i, c_j)
 * (Definition 1).  Every matrix argument is a DEVICE pointer to row-major
 * bit rows: row i starts at word i*ld; column j is bit (j & 63) of word
 * (j >> 6) of that row (least significant bit first).  `ld` (words) must be
 * >= ceil(cols/64).  Bits of columns >= cols ("padding") must be 0 on input
 * (checked when opts->check_padding is set) and are 0 on output, including
 * whole padding words up to ld.  A vector (a partially grounded query
 * r(c, Y), Section 3.3) is a single row; k queries are k rows.
 *
 * ---------------------------------------------------------------- ownership
 * The caller owns every buffer it passes.  The library never frees a caller
 * pointer and keeps none after a call returns.  A handle owns its device
 * workspace (grown on demand, freed by bmlp_destroy).
 *
 * ---------------------------------------------------------------- streams
 * `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 * work of a call is ordered on that stream.  Calls that iterate to a fixpoint
 * read a one-word flag back each iteration and therefore return with the
 * result complete; the element-wise, packing and single-product calls are
 * asynchronous on the stream.
 *
 * ---------------------------------------------------------------- errors
 * Every call returns a bmlp_status.  No C++ exception crosses the ABI.  On
 * error the outputs are unspecified, no other caller memory is written, and
 * bmlp_last_error() (thread-local, valid until the next call on the same
 * thread) describes the failure.  Device faults surface as BMLP_EDEVICE.
 * A handle must not be used by two threads at once.
 */
#ifndef BMLP_H
#define BMLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bmlp_ctx *bmlp_handle;

typedef enum {
  BMLP_OK = 0,
  BMLP_EINVAL = -1,  /* null pointer, negative size, ld too small, bad option, index out of range */
  BMLP_EALIGN = -2,  /* pointer not aligned (8 bytes for bit matrices, 4 for int32 arrays) */
  BMLP_EALIAS = -3,  /* an output overlaps an input */
  BMLP_EPAD = -4,    /* nonzero padding bits in an input (opts->check_padding) */
  BMLP_ENOMEM = -5,  /* workspace allocation failed or would exceed opts->workspace_limit */
  BMLP_EDEVICE = -6, /* HIP runtime error or device fault */
  BMLP_EITER = -7,   /* iteration cap exceeded (Appendix C, Propositions 1-2); indicates a bug */
  BMLP_EMODEL = -8   /* dispatcher model or tuning cache file missing, corrupt or incompatible */
} bmlp_status;

/* Kernel families ("arms").  Every arm returns identical bits. */
typedef enum {
  BMLP_ARM_AUTO = -1,
  BMLP_ARM_PRODUCT_VALU = 0,  /* bit-packed product: LDS-staged 64-bit words, wave AND/OR */
  BMLP_ARM_PRODUCT_MFMA = 1,  /* 4-bit (e2m1) matrix-core product, exact fp32 accumulate, > 0 threshold */
  BMLP_ARM_SMP_DENSE = 2,     /* selection by repeated dense products (semi-naive delta . R1) */
  BMLP_ARM_SMP_SPARSE = 3,    /* selection by sparse-frontier expansion, whole fixpoint per row in one launch */
  BMLP_ARM_SMP_CLOSURE = 4,   /* selection as V . R1+ after BMLP-RMS (closure reuse, Section 4) */
  BMLP_ARM_COMPOSE_RMS = 5,   /* compose: Rs+ by BMLP-RMS, then P = Rb | Rs+ . Rb */
  BMLP_ARM_COMPOSE_SEMINAIVE = 6, /* compose: P^T = Rb^T (Rs^T)*, reflexive selections over the transposed step */
  BMLP_ARM_SMP_SPARSE_ROUNDS = 7, /* selection by rounds, every round by sparse-frontier expansion */
  BMLP_ARM_SMP_ADAPTIVE = 8,  /* selection by rounds, each round's kernel chosen on the device by the model */
  BMLP_ARM_COMPOSE_ROWWISE = 9, /* compose: P[X] = Rb[X] | OR of Rb[Z] over Z in e_X Rs+, only for rows X with
                                  a step edge (selections over Rs, rows of Rb gathered; n <= 131072) */
  BMLP_ARM_PRODUCT_GATHER = 10, /* (in arm traces) a squaring of a sparse R done as row gathers: row i of
                                  R | R.R = R[i] | OR of the rows k over the set bits k of R[i] */
  BMLP_ARM_PRODUCT_SEMINAIVE = 11, /* (in arm traces) a squaring done from the bits D new in the last one:
                                  R | R.R = R | D.R | R.D (D.R by row gathers, R.D by a product over the
                                  nonempty rows of D) */
  BMLP_ARM_PRODUCT_SEMINAIVE_T = 12, /* (in arm traces) the same squaring with R.D = (D^T . R^T)^T, a second
                                  row gather over the bits of D between transposes (D's bits spread over
                                  many rows) */
  BMLP_ARM_SMP_CLOSURE_SELECT = 13 /* selection as V . R1+ with R1+ built by the one-launch selection from
                                  every source (the rows of I . R1+, Eq. 5 with V = I; n <= 131072):
                                  the same closure as BMLP-RMS, by frontier expansion instead of squarings.
                                  Not available in bmlp_batched, whose closures are squared. */
} bmlp_arm;

typedef enum {
  BMLP_DISPATCH_PLAIN = 0,   /* fixed schedule */
  BMLP_DISPATCH_LEARNED = 1, /* learned dispatcher (falls back to plain without a model) */
  BMLP_DISPATCH_FORCED = 2   /* use the arms given in the options */
} bmlp_dispatch;

typedef struct {
  uint32_t size;          /* sizeof(bmlp_opts); set by bmlp_opts_init */
  int32_t dispatch;       /* bmlp_dispatch */
  int32_t product_arm;    /* BMLP_ARM_AUTO, _PRODUCT_VALU or _PRODUCT_MFMA */
  int32_t smp_arm;        /* BMLP_ARM_AUTO, _SMP_DENSE, _SMP_SPARSE, _SMP_CLOSURE, _SMP_SPARSE_ROUNDS,
                             _SMP_ADAPTIVE or _SMP_CLOSURE_SELECT */
  int32_t compose_arm;    /* BMLP_ARM_AUTO, _COMPOSE_RMS, _COMPOSE_SEMINAIVE or _COMPOSE_ROWWISE */
  int32_t rms_variant;    /* 0: R <- R | R.R to a fixpoint (default);
                             1: Algorithm 1 as printed: R = I + R1, square to a fixpoint, times R1 */
  int32_t smp_reflexive;  /* 0: V . R1+ (the paper's answer, default); 1: V . R1* = V | V . R1+ */
  int32_t check_padding;  /* nonzero: validate input padding bits (one extra pass) */
  int64_t workspace_limit;/* bytes of device workspace a call may hold; 0 = unlimited */
} bmlp_opts;

typedef struct {
  int32_t iterations;      /* fixpoint rounds (squarings for RMS, rounds for SMP/compose) */
  int32_t products;        /* launches of the product kernels (incl. Algorithm 1's final product); a
                              squaring done by row gathers counts in iterations and arm_trace only */
  int32_t arm_trace[64];   /* arm used in each round (first 64 rounds); -1 past the end */
  int32_t arm;             /* the arm that served the call */
  int32_t products_mfma;   /* of the timed product launches, those of the matrix-core (MFMA) kernel */
  uint64_t bool_ops;       /* algorithmic Boolean operations: 2*m*k*n per dense (m x k).(k x n) product */
  uint64_t bytes_moved;    /* algorithmic device bytes read + written */
  double device_ms;        /* device time of the call (HIP events on the call's stream) */
  double product_ms;       /* device time inside the product kernels alone (events around each launch) */
  uint64_t product_bool_ops; /* algorithmic Boolean operations of those product launches */
  double product_ms_mfma;    /* the part of product_ms spent in matrix-core (MFMA) product launches */
  uint64_t product_bool_ops_mfma; /* the part of product_bool_ops done by those launches */
  uint64_t mfma_ops_issued;  /* matrix-core operations those launches actually issued: less than their
                                Boolean operations when output tiles are already saturated or words of k
                                are zero across a row block, more on ragged tile edges */
  int32_t gathers;           /* BMLP-RMS squarings done by row gathers (events around each) */
  double gather_ms;          /* device time of those squarings */
  uint64_t gather_bytes;     /* their algorithmic bytes: per squaring of an R with b set bits, the n rows of R
                                read, the b source rows read and the n rows written, n / 8 bytes each */
} bmlp_stats;

/* ------------------------------------------------------------ handles */
/* Create a handle on HIP device `device` (made current for the calls).  */
bmlp_status bmlp_create(bmlp_handle *h, int device);
/* Release the handle and its workspace.  NULL is accepted. */
bmlp_status bmlp_destroy(bmlp_handle h);
/* Thread-local description of the last failure on this thread. */
const char *bmlp_last_error(void);
/* Fill *o with defaults: plain dispatch, automatic arms, default variants. */
void bmlp_opts_init(bmlp_opts *o);
/* Library version as 10000*major + 100*minor + patch. */
int32_t bmlp_version(void);

/* ------------------------------------------------------------ facts -> matrices (Section 3.2) */
/* bits (rows x n, ld) := dense 0/1 bytes (rows x n, row stride ldd >= n); any nonzero byte is 1. */
bmlp_status bmlp_pack_u8(bmlp_handle h, const uint8_t *dense, int64_t rows, int64_t n, int64_t ldd,
                         uint64_t *bits, int64_t ld, void *stream);
/* bits (rows x n, ld) := the m facts (row[e], col[e]) (int32 device arrays; duplicates allowed).
   An index outside [0,rows) x [0,n) gives BMLP_EINVAL.  Synchronises the stream (error check). */
bmlp_status bmlp_pack_coo(bmlp_handle h, const int32_t *row, const int32_t *col, int64_t m, int64_t rows,
                          int64_t n, uint64_t *bits, int64_t ld, void *stream);
/* bmlp_pack_coo without its synchronisation, for streams of small packings: asynchronous on the stream.
   A fact outside [0,rows) x [0,n) is skipped (nothing is written outside `bits`) and latched in the handle;
   bmlp_deferred_error reports it. */
bmlp_status bmlp_pack_coo_async(bmlp_handle h, const int32_t *row, const int32_t *col, int64_t m, int64_t rows,
                                int64_t n, uint64_t *bits, int64_t ld, void *stream);
/* BMLP_EINVAL when a fact given to bmlp_pack_coo_async on this handle since the last check lay outside its
   matrix (the latch is then cleared), else BMLP_OK.  Synchronises the stream. */
bmlp_status bmlp_deferred_error(bmlp_handle h, void *stream);
/* Facts from a bit matrix (decoding, the inverse of bmlp_pack_coo): the set bits of `bits` (rows x n,
   ld) as (row, column) pairs, sorted by row and then column, written to the DEVICE int32 arrays row_out
   and col_out (either may be NULL) of capacity `cap` entries.  *count (HOST) receives the number of
   set bits.  With both outputs NULL only the count is computed (the usual first call); with
   cap < *count nothing is written and BMLP_EINVAL is returned.  Section 3.2 (each matrix row
   encodes the facts r(c_i, c_j) of its set bits). */
bmlp_status bmlp_unpack_coo(bmlp_handle h, const uint64_t *bits, int64_t rows, int64_t n, int64_t ld,
                            int32_t *row_out, int32_t *col_out, int64_t cap, int64_t *count, void *stream);
/* dense (rows x n bytes, stride ldd) := bits; the decoding of a matrix back into facts. */
bmlp_status bmlp_unpack_u8(bmlp_handle h, const uint64_t *bits, int64_t rows, int64_t n, int64_t ld,
                           uint8_t *dense, int64_t ldd, void *stream);

/* ------------------------------------------------------------ operators (Section 2, Section 4) */
/* C = A + B (element-wise OR).  C may equal A or B. */
bmlp_status bmlp_or(bmlp_handle h, const uint64_t *A, const uint64_t *B, uint64_t *C, int64_t rows, int64_t n,
                    int64_t ld, void *stream);
/* C = A AND B (element-wise).  C may equal A or B. */
bmlp_status bmlp_and(bmlp_handle h, const uint64_t *A, const uint64_t *B, uint64_t *C, int64_t rows, int64_t n,
                     int64_t ld, void *stream);
/* C = A AND NOT B (element-wise difference).  C may equal A or B. */
bmlp_status bmlp_andnot(bmlp_handle h, const uint64_t *A, const uint64_t *B, uint64_t *C, int64_t rows, int64_t n,
                        int64_t ld, void *stream);
/* C = NEG(A): every bit of the rows x n matrix flipped; padding stays 0 (Section 3.4, Fig. 3). */
bmlp_status bmlp_not(bmlp_handle h, const uint64_t *A, uint64_t *C, int64_t rows, int64_t n, int64_t ld,
                     void *stream);
/* AT (cols x rows, ldat) = TRANSP(A) (rows x cols, lda): swaps a relation's arguments.
   AT must not overlap A. */
bmlp_status bmlp_transpose(bmlp_handle h, const uint64_t *A, int64_t rows, int64_t cols, int64_t lda,
                           uint64_t *AT, int64_t ldat, void *stream);
/* C = Cold + A x B over the Boolean semiring (Section 2); Cold may be NULL (then C = A x B) and may
   equal C.  A: m x kdim (lda), B: kdim x n (ldb), C: m x n (ldc).  C must not overlap A or B.
   opts may be NULL (defaults); opts->product_arm selects the kernel.  The matrix-core arm keeps its
   sums exact up to kdim = 4,194,304 and returns BMLP_EINVAL beyond (the default choice then takes
   the VALU arm). */
bmlp_status bmlp_product(bmlp_handle h, const uint64_t *A, int64_t lda, const uint64_t *B, int64_t ldb,
                         const uint64_t *Cold, uint64_t *C, int64_t ldc, int64_t m, int64_t kdim, int64_t n,
                         const bmlp_opts *opts, void *stream, bmlp_stats *stats);

/* ------------------------------------------------------------ the BMLP algorithms */
/* BMLP-RMS (Algorithm 1; Eq. 1 fixed point): Rstar = R1+ = sum_{k>=1} R1^k, i.e. Rstar_ij = 1 iff
   a path of length >= 1 leads from i to j.  R1, Rstar: n x n, leading dimension ld.  Rstar must
   not overlap R1.  The default variant iterates R <- R + R x R from R1 (ceil(log2 L)+1 products,
   L the longest shortest path); variant 1 steps Algorithm 1 as printed.  Same bits either way.
   Under the learned schedule (variant 0, n <= 131072) the dispatcher may build the same closure by
   the one-launch selection from every source (Eq. 5 with V = I) where it predicts that cheaper;
   forced with smp_arm BMLP_ARM_SMP_CLOSURE_SELECT it always does; stats->arm then says so. */
bmlp_status bmlp_rms(bmlp_handle h, const uint64_t *R1, uint64_t *Rstar, int64_t n, int64_t ld,
                     const bmlp_opts *opts, void *stream, bmlp_stats *stats);
/* BMLP-SMP (Eq. 5; Algorithm 2): Vstar = V x R1+ row by row, the answers of the k partially
   grounded queries whose constants are the set bits of each row of V (a row with several bits
   answers the union).  V, Vstar: k x n (ldv); R1: n x n (ld).  With opts->smp_reflexive the answer
   is V x R1* = V + V x R1+.  Vstar must not overlap V or R1. */
bmlp_status bmlp_smp(bmlp_handle h, const uint64_t *R1, int64_t n, int64_t ld, const uint64_t *V,
                     uint64_t *Vstar, int64_t k, int64_t ldv, const bmlp_opts *opts, void *stream,
                     bmlp_stats *stats);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): the selection of bmlp_smp, Vstar = V x R1+ (V x R1* when reflexive
   is nonzero), always by the one-launch sparse-frontier kernel, with the relation's edge index (CSR,
   and from mean out-degree 4 the in-edges too) built in a fixed 64 MiB device array of the library
   instead of the handle's workspace.  It calls no hipMalloc, hipFree or allocating routine.  Limits:
   n <= 131072, and the index must fit: about 28 (n + 1) bytes plus 4 bytes per edge (8 per edge from
   mean degree 4); larger inputs give BMLP_ENOMEM with nothing written.  Synchronises the stream once (the
   edge count, read back into the handle's pinned words, sizes the index); the selection itself is
   asynchronous on the stream.  Every call on one device shares that device's array, and its contents
   are those of the last call: calls that overlap on one device (other streams, other threads or other
   handles) race and must not be issued.  Same arguments and errors as bmlp_smp otherwise. */
bmlp_status bmlp_smp_noalloc(bmlp_handle h, const uint64_t *R1, int64_t n, int64_t ld, const uint64_t *V,
                             uint64_t *Vstar, int64_t k, int64_t ldv, int32_t reflexive, void *stream);
/* General linear recursion over binary predicates (Theorem 1): the least model of
       p(X,Y) <- b(X,Y).    p(X,Y) <- s(X,Z), p(Z,Y).
   as P = Rs* x Rb, the least P with P = Rb + Rs x P.  Rbase, Rstep, P: n x n (ld).  P must not
   overlap Rbase or Rstep.  compose_linear(R1, R1) = rms(R1). */
bmlp_status bmlp_compose_linear(bmlp_handle h, const uint64_t *Rbase, const uint64_t *Rstep, uint64_t *P,
                                int64_t n, int64_t ld, const bmlp_opts *opts, void *stream, bmlp_stats *stats);

/* Two-sided linear recursion
       p(X,Y) <- b(X,Y).    p(X,Y) <- l(X,X1), p(X1,Y1), r(Y1,Y).
   as the least P with P = Rbase + Rleft x P x Rright, i.e. P = sum over k >= 0 of Rleft^k Rbase
   Rright^k (same-generation when l = up and r = down; a multilinear extension the paper names as
   future work).  Semi-naive rounds; stats->iterations is the number of rounds.  Rbase, Rleft, Rright,
   P: n x n (ld); P must not overlap the others.  With Rright = I this is compose_linear(Rbase, Rleft);
   with Rleft = I it is Rbase x Rright*. */
bmlp_status bmlp_compose_two_sided(bmlp_handle h, const uint64_t *Rbase, const uint64_t *Rleft,
                                   const uint64_t *Rright, uint64_t *P, int64_t n, int64_t ld,
                                   const bmlp_opts *opts, void *stream, bmlp_stats *stats);

/* Closure under insertions: Rplus (n x n, ld) holds T = R1+ of some relation R1 on entry (the caller's
   promise; it is not checked) and (R1 | E)+ on return, where E is the b edges (src[i], dst[i]).
   Closures only grow under insertions (dynamic databases, named as future work in the paper's
   conclusion), so with U = T | I the new paths are x ->U src_i -> dst_i ->U ... -> dst_j ->U y, and
   (R1 | E)+ = T | A . M* . B with A = columns src_i of U, B = rows dst_j of U and
   M[i][j] = U[dst_i][src_j] (b x b).  src, dst: DEVICE int32 arrays of b indices in [0, n)
   (BMLP_EINVAL otherwise, Rplus unchanged); duplicate and already-implied edges are fine.  b = 0 is a
   no-op.  Uses handle workspace of about 3 b n / 8 + 2 n b / 8 bytes plus that of a b x b closure.
   stats: the products and the small closure, as for the other calls. */
bmlp_status bmlp_closure_insert(bmlp_handle h, uint64_t *Rplus, int64_t n, int64_t ld, const int32_t *src,
                                const int32_t *dst, int64_t b, const bmlp_opts *opts, void *stream,
                                bmlp_stats *stats);

/* ------------------------------------------------------------ batches of graphs */
/* One graph of a batch: its relation, where its closure goes, and its query rows. */
typedef struct {
  int64_t n;              /* constants (nodes) of this graph; 0 is allowed */
  int64_t ld;             /* leading dimension of R1 (words) */
  const uint64_t *R1;     /* n x n relation (device) */
  uint64_t *closure;      /* out: n x n R1+ with leading dimension ldc, or NULL */
  int64_t ldc;            /* leading dimension of closure (ignored when closure is NULL) */
  int64_t k;              /* query rows (0 for none) */
  int64_t ldv;            /* leading dimension of V and Vstar */
  const uint64_t *V;      /* k x n query rows (device) */
  uint64_t *Vstar;        /* out: k x n answers V x R1+ */
} bmlp_graph_desc;

/* BMLP-RMS and BMLP-SMP (Section 3.3, Eqs. 4-5; Algorithms 1-2) for `count` independent graphs of
   any sizes in one hipGraph launch: for each graph the closure R1+ and the answers V x R1+ (read off
   the closure, the reuse of intermediate results of Section 4).  `graphs` is a host array; the
   device buffers it points to must not overlap each other across outputs and inputs.  The launch is
   asynchronous on `stream` (the captured graph is cached on the handle and reused while the
   descriptors stay the same); with `stats` non-NULL the call waits and fills it.  Graph outputs of
   different descriptors must not overlap. */
bmlp_status bmlp_batched(bmlp_handle h, const bmlp_graph_desc *graphs, int32_t count, const bmlp_opts *opts,
                         void *stream, bmlp_stats *stats);

/* ------------------------------------------------------------ sessions over one relation */
/* A session answers a stream of selections over one relation R1 (n x n, ld; the caller keeps it
   alive and unchanged while the session is open).  It keeps the relation's CSR and statistics and,
   once computed, its closure R1+, so that later queries are answered by reading rows of the closure
   (reuse of intermediate results, Section 4).  Under the plain schedule a session never computes
   the closure; under the learned schedule it does so when the model's predicted cost of the
   closure falls below the time already spent answering this relation's queries iteratively
   (ski-rental rule), and builds it by BMLP-RMS or by the selection from every source
   (BMLP_ARM_SMP_CLOSURE_SELECT), whichever the model predicts cheaper.  Forced with smp_arm
   BMLP_ARM_SMP_CLOSURE or _SMP_CLOSURE_SELECT, the first query builds the closure that way.  The
   session owns its closure buffer (n x ceil(n/64) words). */
typedef struct bmlp_graph_s *bmlp_graph;
bmlp_status bmlp_graph_open(bmlp_handle h, const uint64_t *R1, int64_t n, int64_t ld, void *stream, bmlp_graph *g);
/* Vstar = V x R1+ (Eq. 5), like bmlp_smp; stats->arm tells which arm answered.  Without stats the query
   is asynchronous on the stream except where the learned schedule times it (before the closure exists). */
bmlp_status bmlp_graph_query(bmlp_graph g, const uint64_t *V, uint64_t *Vstar, int64_t k, int64_t ldv,
                             const bmlp_opts *opts, void *stream, bmlp_stats *stats);
/* The k one-hot queries r(src[i], Y) (Eq. 5 with a single source each): Vstar row i = e_src[i] x R1+
   (| e_src[i] when opts->smp_reflexive), like bmlp_graph_query with the query rows given by their
   sources (DEVICE int32 array).  Once the session holds the closure an answer is one closure row, read
   by index.  An index outside [0, n) gives an all-zero answer row and is latched for
   bmlp_deferred_error (no synchronisation).  Without stats the query is asynchronous on the stream
   except where the learned schedule times it (before the closure exists). */
bmlp_status bmlp_graph_query_sources(bmlp_graph g, const int32_t *src, uint64_t *Vstar, int64_t k, int64_t ldv,
                                     const bmlp_opts *opts, void *stream, bmlp_stats *stats);
/* Whether the session holds the closure (1) or not (0). */
int32_t bmlp_graph_has_closure(bmlp_graph g);
/* The arm (bmlp_arm) that served the session's last query, -1 before the first; host-side, no waiting.
   The query that built the closure reports the build (BMLP_ARM_SMP_CLOSURE: by BMLP-RMS,
   _SMP_CLOSURE_SELECT: by selection); later answers read off it report BMLP_ARM_SMP_CLOSURE. */
int32_t bmlp_graph_last_arm(bmlp_graph g);
bmlp_status bmlp_graph_close(bmlp_graph g);

/* ------------------------------------------------------------ autotuned tile code */
/* Several kernels come in candidate versions ("tile code": tile shapes, words of k per LDS stage, the
   order of output tiles over the XCDs, rows per wave); every candidate returns identical bits, they
   differ in speed only.  A handle keeps, per tuned kernel and size/density bucket, the candidate to
   use (-1: the built-in default).  Tuned kernels:
     BMLP_TUNE_MFMA_PRODUCT  the matrix-core product (BMLP_ARM_PRODUCT_MFMA)
     BMLP_TUNE_VALU_PRODUCT  the bit-packed VALU product (BMLP_ARM_PRODUCT_VALU)
   Buckets of a product (m x kdim).(kdim x n): 4 * size + class, size 0..3 by the dense operation
   count 2 m kdim n (below about 2 x 2048^3, 2 x 4096^3, 2 x 8192^3, beyond), class 0..3 by the left
   operand: set bits below 1/4096, below 1/64, denser or unknown, block-structured (the squarings of a
   relabelled relation).  bmlp_create loads $BMLP_AUTOTUNE_CACHE, else autotune_cache.json beside the
   library, when it exists and was written on the same kind of device. */
typedef enum { BMLP_TUNE_MFMA_PRODUCT = 0, BMLP_TUNE_VALU_PRODUCT = 1 } bmlp_tune_kernel;
#define BMLP_TUNE_MAX_CANDIDATES 8
/* Number of candidates / buckets of a tuned kernel (0 for an unknown kernel). */
int32_t bmlp_tune_candidates(int32_t kernel);
int32_t bmlp_tune_buckets(int32_t kernel);
/* The bucket of a product of the given shape and left-operand density (density < 0: unknown;
   structured nonzero: block-structured), or -1. */
int32_t bmlp_tune_bucket_of(int32_t kernel, int64_t m, int64_t kdim, int64_t n, double density, int32_t structured);
/* The handle's candidate for (kernel, bucket) (-1: default) and the device time it was chosen with
   (ms; 0 when set by hand or not measured); ms may be NULL. */
bmlp_status bmlp_tune_get(bmlp_handle h, int32_t kernel, int32_t bucket, int32_t *variant, float *ms);
/* Pin a candidate (-1: back to the default) for one bucket, or for every bucket with bucket = -1. */
bmlp_status bmlp_tune_set(bmlp_handle h, int32_t kernel, int32_t bucket, int32_t variant);
/* Run the autotuner on the handle's device: for every kernel in kernel_mask (bit k = tuned kernel k) and
   every bucket, time each candidate `reps` times (after one warm-up launch; the median counts) on seeded
   synthetic squarings C = A | A.A at the bucket's representative size (n = 2048, 4096, 8192, 16384) and
   class, and keep the fastest.  Takes a few seconds and up to 3 x 32 MiB of workspace.  With cache_out
   non-NULL the result is written there (JSON, see bmlp_tune_save).  report (nullable, host) receives
   kernels x buckets x BMLP_TUNE_MAX_CANDIDATES median times in ms (-1 where not measured). */
bmlp_status bmlp_autotune(bmlp_handle h, int32_t kernel_mask, int32_t reps, const char *cache_out, float *report);
/* Write the handle's choices to / read them from a JSON tuning cache keyed by the device's architecture
   name and compute-unit count.  A cache of another kind of device, or a malformed one, gives
   BMLP_EMODEL and leaves the handle unchanged. */
bmlp_status bmlp_tune_save(bmlp_handle h, const char *path);
bmlp_status bmlp_tune_load(bmlp_handle h, const char *path);

/* ------------------------------------------------------------ the learned dispatcher */
/* The dispatcher is a small FP32 network (16 features -> 64 -> 64 -> 4 outputs, ReLU) predicting
   the log device time (ms) of kernel arms.  Outputs mean, for a round-level query (feature 8 = 0):
   [0] one round by the dense product, [1] one round by sparse-frontier expansion; for a call-level
   query (feature 8 = 1): [0] the whole selection by rounds, [2] by the closure, [3] by the
   one-launch sparse-frontier kernel.  It chooses kernels only; every arm returns the same bits. */
typedef struct {
  int32_t rounds;             /* rounds recorded (at most 64) */
  int32_t call_arm;           /* arm that served the call */
  int32_t arm[64];            /* arm of each round (BMLP_ARM_SMP_DENSE or _SMP_SPARSE) */
  float round_ms[64];         /* device time of each round */
  float features[64][16];     /* round-level features at the start of each round */
  float call_features[16];    /* call-level features */
  float pred[64][4];          /* model outputs per round (learned schedule) */
  float call_pred[4];         /* model outputs for the call decision (learned schedule) */
  float total_ms;             /* device time of the whole call */
} bmlp_trace;
/* Record per-round features and timings of subsequent selection calls into *trace (owned by the
   caller; NULL stops recording).  Recording synchronises after every round. */
bmlp_status bmlp_set_trace(bmlp_handle h, bmlp_trace *trace);
/* Load / save the dispatcher model (versioned header + CRC-32).  A missing, corrupt or mismatched
   file gives BMLP_EMODEL and leaves the handle's model unchanged; without a model the learned
   schedule falls back to the plain one. */
bmlp_status bmlp_dispatcher_load(bmlp_handle h, const char *path);
bmlp_status bmlp_dispatcher_save(bmlp_handle h, const char *path);
/* 1 when the handle has a model. */
int32_t bmlp_dispatcher_loaded(bmlp_handle h);
/* Train the handle's model on the GPU (hand-written forward, backward and Adam kernels), full batch:
   X rows x 16 features, T rows x 4 targets (log ms), M rows x 4 mask (1 = target present); host
   arrays.  Inputs are standardised with the data's mean and deviation, parameters initialised from
   `seed`.  *loss_out receives the final masked mean-squared error. */
bmlp_status bmlp_dispatcher_train(bmlp_handle h, const float *X, const float *T, const float *M, int64_t rows,
                                  int32_t epochs, float lr, uint64_t seed, float *loss_out);
/* Y (rows x 4) = model outputs for X (rows x 16); host arrays, GPU compute. */
bmlp_status bmlp_dispatcher_forward(bmlp_handle h, const float *X, int64_t rows, float *Y);
/* One forward and backward pass on the GPU with the given parameters (5,508 floats in the layout
   W1[64][16] b1[64] W2[64][64] b2[64] W3[4][64] b3[4]) and standardisation (mu, sd: 16 each):
   *loss = masked mean-squared error, grad (5,508) = its gradient.  Host arrays. */
bmlp_status bmlp_mlp_loss_grad(bmlp_handle h, const float *params, const float *mu, const float *sd, const float *X,
                               const float *T, const float *M, int64_t rows, float *loss, float *grad);

#ifdef __cplusplus
}
#endif

#endif /* BMLP_H */
