/*
 * polyspec.h -- C ABI of the MI355X (gfx950) polyspectrum estimator library.
 *
 * The library computes the angle-averaged n-point polyspectrum of a real field
 * on a periodic N^3 grid with the FFT form of the estimator of Tomlinson, Jeong &
 * Kim (2019) (Sec. 2: the Fourier representation of the Dirac delta turns the sum
 * over closed n-gons into a grid sum of products of shell-filtered inverse
 * transforms; Appendix A: unnormalised DFTs and the polygon-count normalisation
 * obtained by running the same estimator on unit shells).
 *
 * Conventions shared by every call:
 *  - delta_hat[q] is the unnormalised forward DFT (sum_x delta[x] e^{-2 pi i q.x/N});
 *    shell fields d_s[x] = sum_q [s(q) = s] delta_hat[q] e^{+2 pi i q.x/N}.
 *  - Shell s = 1..n_shells of width D (units of the fundamental wavenumber k_f)
 *    holds the modes with (s - 1/2) D <= |q| < (s + 1/2) D, decided exactly on the
 *    integer |q|^2.  The DC mode is in no shell.
 *  - Tuples are sorted t_1 <= ... <= t_n, lexicographic with t_n fastest (the
 *    paper's k_1 >= ... >= k_n row-major order, each tuple reversed).  Only tuples
 *    that close (polygon count n_t > 0) are reported; n_closing is their number.
 *  - B_t = f * S_t / (N^3 n_t) with S_t = sum_x prod_j d_{t_j}[x] and f = 1, or
 *    f = V^{n-1} / N^{3n}, V = L^3, when box_length L > 0 (Appendix A).
 *  - Every device pointer is caller-owned and must stay valid until the stream
 *    work that uses it has finished.  Arrays are dense, row-major, last index
 *    fastest.  Real fields are float32 [batch][N][N][N].
 *  - Every call returns a status; none throws, aborts or exits.  A failed call
 *    leaves the plan as it was, and polyspec_last_error() gives detail text.
 *  - All work is enqueued on the plan's stream (a hipStream_t passed as void*,
 *    NULL for the default stream) and is asynchronous unless stated otherwise.
 *  - A plan is not thread-safe; use one plan per host thread.
 */
#ifndef POLYSPEC_H
#define POLYSPEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct polyspec_plan_s* polyspec_plan_t;

typedef enum {
  POLYSPEC_OK = 0,
  POLYSPEC_ERR_INVALID_ARG = 1,        /* bad descriptor field, null pointer, size mismatch */
  POLYSPEC_ERR_ALIASING = 2,           /* order * (n_shells + 1/2) * width > N without ALLOW_ALIASING */
  POLYSPEC_ERR_OUT_OF_MEMORY = 3,      /* device or host allocation failed */
  POLYSPEC_ERR_DEVICE = 4,             /* a HIP runtime call or kernel launch failed */
  POLYSPEC_ERR_COUNT_NOT_INTEGRAL = 5, /* a count quotient q missed an integer by max(1e-3, |q| 2^-46) */
  POLYSPEC_ERR_STATE = 6,              /* call out of order (contract before shells, ...) */
  POLYSPEC_ERR_UNSUPPORTED = 7         /* valid request outside what this build implements */
} polyspec_status;

/* Arithmetic of the product-sum contraction.  Shell fields are always float32 and
 * sums across grid tiles are always float64.  SPLIT_* carry each float32 operand as
 * hi + lo of a 16-bit type and form hi*hi + hi*lo + lo*hi on the matrix cores,
 * accumulating in float32.  SPLIT_FP16 scales every shell by a power of two so that
 * its largest magnitude lies in [2^6, 2^7); the scale is removed exactly in float64.
 * (Not in the paper: a precision extension of its product-and-sum step.) */
typedef enum {
  POLYSPEC_FP32 = 0,
  POLYSPEC_SPLIT_BF16 = 1,
  POLYSPEC_SPLIT_FP16 = 2
} polyspec_precision;

enum {
  POLYSPEC_INPUT_HALF_SPECTRUM = 1u, /* polyspec_shells input is delta_hat, complex64 [batch][N][N][N/2+1] */
  POLYSPEC_ALLOW_ALIASING = 2u,      /* accept order*(n_shells+1/2)*width > N: exact mod-N estimator */
  POLYSPEC_NAN_GUARD = 8u,           /* contract reports POLYSPEC_ERR_DEVICE on a non-finite output */
  POLYSPEC_STREAM_SLABS = 16u,       /* shell fields are never stored whole: see polyspec_set_slab_planes */
  POLYSPEC_MULTIPOLE = 32u           /* order 3: bispectrum multipoles about the third axis, see polyspec_set_multipole */
};

typedef struct {
  int32_t N;            /* grid points per side; a power of two, 32 <= N <= 1024            */
  int32_t order;        /* n = 2 to 6 (Sec. 4.2 runs the estimator up to hexagons, n = 6)  */
  int32_t n_shells;     /* N_b >= 1; (N_b + 1/2) * width <= N/2; the matrix-core contraction
                           handles N_b <= 128 at orders 2 to 4 and N_b <= 32 at orders 5 and 6;
                           polyspec_backward needs N_b <= 64 (orders 3 and 4)   */
  double shell_width;   /* D > 0, in units of k_f (exact binary value is used)              */
  int32_t batch;        /* independent fields processed together, >= 1                      */
  int32_t precision;    /* polyspec_precision                                                */
  double box_length;    /* L; 0 => estimator units S/(N^3 n_t); > 0 => times V^{n-1}/N^{3n} */
  uint32_t flags;       /* POLYSPEC_* flags above                                            */
} polyspec_desc;

/* Builds a plan for one geometry (Sec. 2 estimator; Appendix A counts).
 * Validates the descriptor, builds the shell, tuple and tile tables, and computes
 * the polygon counts n_t of every candidate tuple on the device in float64 (the
 * estimator applied to unit shells, Sec. 4 and Appendix A).  Synchronises the
 * stream once to read the counts back.  The count sums are accumulated with
 * compensated (double-double) additions; returns POLYSPEC_ERR_COUNT_NOT_INTEGRAL if
 * any count quotient q misses an integer by max(1e-3, |q| 2^-46) or more, or if a
 * count reaches 2^44.  *out receives the plan. */
polyspec_status polyspec_plan(const polyspec_desc* desc, void* stream, polyspec_plan_t* out);

/* Shell fields (Sec. 2, I_k(x); Appendix A, FFTW(I~)).  d_delta is a device
 * pointer to float32 [batch][N][N][N] (or complex64 [batch][N][N][N/2+1] with
 * POLYSPEC_INPUT_HALF_SPECTRUM).  Computes delta_hat on the ball of modes in any
 * shell, then every d_s, and keeps them in the plan's workspace for contract and
 * backward.  Asynchronous; d_delta may be reused once the stream has passed it. */
polyspec_status polyspec_shells(polyspec_plan_t plan, const void* d_delta);

/* Product sums and normalisation (Sec. 2, the grid sum of products of the I_k;
 * Appendix A, division by N^3 and by the polygon count).  Writes B_t as float64
 * [batch][n_closing] to d_out, and the raw sums S_t (float64, same shape) to
 * d_raw_sums when it is not NULL.  The sums are matrix-core products of row
 * products of the shell fields: shell x shell (n = 2), pair x shell (3), pair x
 * pair (4), pair x triple (5) and triple x triple (6).  POLYSPEC_ERR_STATE before
 * polyspec_shells. */
polyspec_status polyspec_contract(polyspec_plan_t plan, double* d_out, double* d_raw_sums);

/* Adjoint of shells + contract (not in the paper): given dL/dB_t in d_grad_out
 * (float64 [batch][n_closing]), writes the gradient with respect to the input of the
 * last polyspec_shells call, in the same space, to d_grad_delta:
 *  - real-space plans: dL/d delta as float32 [batch][N][N][N];
 *  - POLYSPEC_INPUT_HALF_SPECTRUM plans: complex64 [batch][N][N][N/2+1] holding
 *    dL/dRe delta_hat + i dL/dIm delta_hat.  An entry with q2 = 0 is read once by
 *    the inverse real transform and an entry with 0 < q2 < N/2 twice (itself and its
 *    conjugate mirror), so the entry is g[q] resp. 2 g[q] with g as below; entries
 *    outside every shell are zero.
 * Each position of a closing tuple contributes dL/dB_t f/(N^3 n_t) times the
 * product of the other shell fields to a_m of its shell m; g[q] = sum_m [s(q) = m]
 * R2C(a_m)[q] and dL/d delta is its unnormalised C2R.  Uses the shell fields of
 * the last polyspec_shells call; the caller must not have called polyspec_shells
 * with another input in between (the library cannot tell).  Orders 3 and 4 with at
 * most 64 shells (not multipole plans); POLYSPEC_ERR_UNSUPPORTED otherwise.  The adjoint
 * product runs in float32 for POLYSPEC_FP32 and in split precision otherwise. */
polyspec_status polyspec_backward(polyspec_plan_t plan, const double* d_grad_out, void* d_grad_delta);

/* polyspec_shells followed by polyspec_contract, allocating nothing: for callers that
 * cannot allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid it).  The workspace is the library's static scratch, a
 * file-scope device array of POLYSPEC_STATIC_SCRATCH_BYTES held on each GPU the library
 * runs on until the process ends (its address is looked up when a plan is made).  Plans
 * whose workspace (polyspec_workspace_size) is larger are refused with
 * POLYSPEC_ERR_UNSUPPORTED; the call must run with the plan's device current
 * (POLYSPEC_ERR_INVALID_ARG otherwise).  Inputs and outputs are as for polyspec_shells
 * and polyspec_contract.  The plan's own workspace and the shell fields kept in it are
 * left as they were, so polyspec_backward still refers to the last polyspec_shells call.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one GPU (two
 * streams, two host threads) race and must be serialised by the caller.  Event timing
 * (polyspec_profile) does not cover this call. */
#define POLYSPEC_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
polyspec_status polyspec_forward_static(polyspec_plan_t plan, const void* d_delta, double* d_out,
                                        double* d_raw_sums);

/* Redshift-space bispectrum multipoles (Sec. 5: the estimator on multipole-weighted
 * fields).  A plan made with POLYSPEC_MULTIPOLE (order 3, at most 64 shells, not
 * streamed) has one output tuple (u, v, w), u <= v, for each closing triangle and each
 * distinct choice of its weighted side w; polyspec_tuples lists them (w last) in
 * lexicographic order with the triangle's count.  With the line of sight along the
 * third grid axis and mu = q2 / |q|, the output is
 *   B_ell(u, v; w) = (2 ell + 1) f sum_x d_u d_v d^ell_w / (N^3 n_t),
 * d^ell_w the shell field of delta_hat L_ell(mu).  The plan keeps 2 N_b fields (the
 * shells, then their weighted copies; polyspec_fields returns both).  ell: even, 0 to
 * 16 (odd ell would make the weighted fields imaginary); 0 until set.  Setting it
 * invalidates the fields: call polyspec_shells again.  POLYSPEC_ERR_STATE for a plan
 * without the flag; polyspec_backward is not available for these plans. */
polyspec_status polyspec_set_multipole(polyspec_plan_t plan, int32_t ell);

/* Bytes of device workspace the plan needs for shells, contract and backward. */
polyspec_status polyspec_workspace_size(polyspec_plan_t plan, size_t* bytes);

/* Hands the plan caller-owned device memory of at least polyspec_workspace_size()
 * bytes (256-byte aligned).  Must precede the first polyspec_shells call; without
 * it the plan allocates its own on first use and frees it in polyspec_destroy. */
polyspec_status polyspec_set_workspace(polyspec_plan_t plan, void* d_ptr, size_t bytes);

/* Streamed mode (plans made with POLYSPEC_STREAM_SLABS; the grid is processed in slabs
 * as the paper distributes it over processes, Sec. 3, so that the grids of Sec. 4.3
 * fit).  Storing every shell field takes batch * n_shells * N^3 * 4 bytes (275 GB at
 * N = 1024 with 64 shells), more than one GPU holds.  A streamed plan keeps only the ball of delta_hat and the first
 * inverse pass (O(n_shells N^2 K) values); polyspec_contract then runs the last two
 * inverse passes and the contraction one slab of `planes` x1-planes at a time and adds
 * each slab's sums in float64, in slab order.  The fields are recomputed by every
 * polyspec_contract call; when the contraction scales its operands (FP16 split, orders
 * 5 and 6) each slab takes its own per-field maxima, and the float64 reduction of the
 * slab removes the scale.  polyspec_backward runs slab by slab as well: each slab's
 * fields are made once more, its adjoint product and the adjoint's x2 and x0
 * transforms follow, and the x1 transform and the gradient's inverse passes run once
 * at the end.  polyspec_fields is not available on such plans.
 * polyspec_set_slab_planes sets the slab: a power of two between the smallest slab the
 * last pass accepts (4 at N = 32, 1 above) and N; it must precede the first use of the
 * workspace (POLYSPEC_ERR_STATE after it, or on a plan without the flag).  The default
 * is the largest slab whose fields take at most 2 GiB.  polyspec_slab_planes reports the
 * slab (N for a plan without the flag). */
polyspec_status polyspec_set_slab_planes(polyspec_plan_t plan, int32_t planes);
polyspec_status polyspec_slab_planes(polyspec_plan_t plan, int32_t* planes);

/* Switches the contraction arithmetic (polyspec_precision) for later calls. */
polyspec_status polyspec_set_precision(polyspec_plan_t plan, int32_t precision);

/* Host copies of the closing tuples and their counts.  *n_closing is always set;
 * h_bins (int32 [n_closing][order]) and h_counts (int64 [n_closing]) are filled
 * when not NULL.  Synchronous, touches no device memory. */
polyspec_status polyspec_tuples(polyspec_plan_t plan, int64_t* n_closing, int32_t* h_bins,
                                int64_t* h_counts);

/* Every candidate tuple examined at plan time (sorted tuples that pass the
 * triangle-type bound, or all sorted tuples when aliasing is allowed) with the
 * float64 quotient C_t / N^3 whose rounding gave its count.  Same conventions
 * as polyspec_tuples. */
polyspec_status polyspec_candidates(polyspec_plan_t plan, int64_t* n_candidates, int32_t* h_bins,
                                    double* h_quotients);

/* Device pointer to the kept float32 shell fields [batch][n_shells][N][N][N]
 * (owned by the plan, valid until the next polyspec_shells or polyspec_destroy),
 * for inspection.  POLYSPEC_ERR_STATE before polyspec_shells. */
polyspec_status polyspec_fields(polyspec_plan_t plan, const float** d_fields);

/* Kernel timing.  Phases of polyspec_shells, polyspec_contract and
 * polyspec_backward, one kernel each, in launch order. */
enum {
  POLYSPEC_PH_INPUT_Q3 = 0,   /* input transform, rows x2 -> q2            */
  POLYSPEC_PH_INPUT_Q2,       /* input transform, x0 -> q0                  */
  POLYSPEC_PH_INPUT_Q1,       /* input transform, x1 -> q1 into the ball    */
  POLYSPEC_PH_SHELL_P1,       /* shell fields, masked q1 -> x1              */
  POLYSPEC_PH_SHELL_P2,       /* shell fields, q0 -> x0                     */
  POLYSPEC_PH_SHELL_P3,       /* shell fields, q2 -> x2 complex-to-real     */
  POLYSPEC_PH_CONTRACT,       /* matrix-core product sums per grid chunk    */
  POLYSPEC_PH_REDUCE,         /* float64 sum over grid chunks               */
  POLYSPEC_PH_GATHER,         /* tuple gather and normalisation             */
  POLYSPEC_PH_ADJ_WEIGHTS,    /* adjoint: weights W[m][pair]                */
  POLYSPEC_PH_ADJ_GEMM,       /* adjoint: a_m = W (d_u d_v)                 */
  POLYSPEC_PH_ADJ_Q3,         /* adjoint: rows x2 -> q2                     */
  POLYSPEC_PH_ADJ_Q2,         /* adjoint: x0 -> q0                          */
  POLYSPEC_PH_ADJ_Q1,         /* adjoint: x1 -> q1, shell-masked merge      */
  POLYSPEC_PH_GRAD_P1,        /* gradient field, q1 -> x1                   */
  POLYSPEC_PH_GRAD_P2,        /* gradient field, q0 -> x0                   */
  POLYSPEC_PH_GRAD_P3,        /* gradient field, q2 -> x2 complex-to-real   */
  POLYSPEC_N_PHASES
};

/* Turns event timing of every kernel launch on (enable != 0) or off.  Timing adds
 * a pair of HIP events per launch on the plan's stream and nothing else. */
polyspec_status polyspec_profile(polyspec_plan_t plan, int32_t enable);

/* Waits for the plan's stream, then writes the milliseconds spent in each phase
 * (h_ms, double [POLYSPEC_N_PHASES]) and the number of timed launches (h_launches,
 * int64 [POLYSPEC_N_PHASES], may be NULL) since the last read, and resets them. */
polyspec_status polyspec_profile_read(polyspec_plan_t plan, double* h_ms, int64_t* h_launches);

/* Matrix-core flops that one call issues in a phase, for the plan's current
 * precision: every launched tile counts in full, including entries no tuple
 * needs, so this is the work the hardware does rather than the algorithmic
 * 2 flops per tuple and grid point.  Phases POLYSPEC_PH_CONTRACT and
 * POLYSPEC_PH_ADJ_GEMM (orders 3 and 4) have matrix-core work; every other phase gives 0.
 * Host-only; no device work. */
polyspec_status polyspec_issued_flops(polyspec_plan_t plan, int32_t phase, double* flops);

/* Releases the plan and everything it allocated (not caller workspace).  Waits for
 * the plan's stream.  NULL is accepted. */
polyspec_status polyspec_destroy(polyspec_plan_t plan);

const char* polyspec_status_string(polyspec_status st);

/* Detail of the last failure on this plan (or of the last failed polyspec_plan when
 * plan is NULL); valid until the next call on the same plan. */
const char* polyspec_last_error(polyspec_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* POLYSPEC_H */
