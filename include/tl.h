/*
 * tl.h -- C ABI of libtl.so: FP64 per-grid-point tensor expressions on AMD
 * MI355X (gfx950), after Lewis & Pfeiffer, "Automatic generation of CUDA code
 * performing tensor manipulations using C++ expression templates"
 * (arXiv:1804.10120).
 *
 * Fields.  A tensor field with C independent components over n grid points is
 * one FP64 device buffer laid out component-major: component c of point p is
 * at ptr[c*ld + p], with ld >= n (the paper's one array per tensor component,
 * Sec. 2.1-2.2, made contiguous: one base pointer plus a leading dimension
 * instead of a table of per-component pointers).  Component orders:
 *
 *   symmetric pair (i,j), i <= j  ->  s(i,j): 00->0 01->1 02->2 11->3 12->4 22->5
 *     (the order of the paper's symmetric tensor-index loops, Sec. 2.4)
 *   g, ginv, K, dtg, w    6   s(i,j)
 *   dg                   18   k*6 + s(i,j)   = d_k g_ij
 *   gamma                18   i*6 + s(j,k)   = Gamma^i_jk  (symmetric in jk)
 *   beta                  3   i              = beta_i
 *   dbeta                 9   j*3 + i        = d_j beta_i
 *   nabla_beta            9   j*3 + i        = nabla_j beta_i
 *   alpha                 1   (ld is ignored)
 *
 * Ownership.  The caller owns every buffer; the plain entry points allocate
 * nothing.  All pointers are device pointers (or host pointers of memory the
 * device can access) of 8-byte aligned FP64 data.
 *
 * Execution.  Every compute call is asynchronous on `stream` (a hipStream_t;
 * NULL = the null stream) and performs no host synchronisation; data stays on
 * the device between calls.
 *
 * Errors.  Argument errors are detected before anything is launched and are
 * returned synchronously: a NULL pointer while n > 0 (TL_ERR_NULL); n < 0 or
 * ld < n (TL_ERR_SIZE); a pointer that is not 8-byte aligned (TL_ERR_ALIGN);
 * an output that shares an element with an input or another output
 * (TL_ERR_ALIAS; fields interleaved in one buffer without sharing an element,
 * such as point ranges of one large field, are accepted, and inputs may
 * overlap each other); an invalid tuning or plan argument (TL_ERR_INVALID).
 * A launch failure reported by the HIP runtime returns TL_ERR_HIP.  For every
 * error a message is available from tl_last_error() (per calling thread).
 * n == 0 returns TL_OK without launching.  Numerical conditions are not
 * reported: a singular metric propagates IEEE inf/NaN.  No C++ exception
 * crosses this interface.  Stateless calls are thread-safe; a batch plan must
 * not be used from two threads at once.
 */
#ifndef TL_H
#define TL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TL_ABI_VERSION 4

typedef enum {
  TL_OK = 0,
  TL_ERR_NULL = 1,
  TL_ERR_SIZE = 2,
  TL_ERR_ALIAS = 3,
  TL_ERR_ALIGN = 4,
  TL_ERR_HIP = 5,
  TL_ERR_INVALID = 6
} tl_status;

/* Input field [ncomp][ld] and output field [ncomp][ld]. */
typedef struct { const double* ptr; int64_t ld; } tl_cfield;
typedef struct { double* ptr; int64_t ld; } tl_field;

/* Launch tuning.  A NULL tl_tune* selects the measured default shape, which
 * depends on the kernel and on n.  In a supplied tl_tune a zero block, ppt or
 * grid_mult selects the default value of that member; flags are taken as
 * given.
 *   block      threads per block: 64, 128, 256, 512 or 1024
 *   ppt        consecutive grid points per thread: 1, 2 or 4 (2 and 4 use
 *              16-byte loads and stores and need every field 16-byte aligned
 *              with an even ld; otherwise the call silently uses 1).  4 is
 *              taken by bodies with at most 24 component streams read and
 *              written per point (tl_sym_inverse, tl_dtg, the expressions
 *              assign1, assign2, add1-add3, mult1 and kij, and generated
 *              kernels of that size); the others silently use 2.
 *              tl_christoffel with lanes > 1 ignores ppt.
 *   flags      TL_TUNE_NT: non-temporal (streaming) loads and stores;
 *              TL_TUNE_XCD: the blocks resident on one XCD (workgroups go to
 *              the 8 XCDs round-robin) take consecutive tiles, so each XCD
 *              streams through contiguous address ranges;
 *              TL_TUNE_PTR64: address every component with a 64-bit pointer.
 *              Without it, a call whose fields each span less than 4 GiB
 *              and that uses TL_TUNE_NT addresses them through one buffer
 *              descriptor per field and 32-bit offsets (fewer instructions
 *              per access; the results are identical)
 *   grid_mult  0: one tile of block*ppt points per block; k > 0: a persistent
 *              grid of k blocks per compute unit striding over the tiles
 *   lanes      lanes per grid point, 0 or 1 (one lane computes all components
 *              of its point) or, for tl_christoffel only, 2, 3, 6, 9 or 18:
 *              the 18 stored components of a point are spread over that many
 *              neighbouring lanes (lane r of a point stores the components
 *              q with q mod lanes == r; every lane loads the point's inputs),
 *              the paper's parallelisation over left-hand-side components.
 *              ppt and grid_mult are then ignored; results agree with the
 *              one-lane kernel's to rounding.
 *              Other values, or lanes > 1 for another entry point:
 *              TL_ERR_INVALID.                                              */
typedef struct { int32_t block, ppt, flags, grid_mult, lanes; } tl_tune;
#define TL_TUNE_NT 1
#define TL_TUNE_XCD 2
#define TL_TUNE_PTR64 4

/* ---- Unfused steps ------------------------------------------------------ */

/* Inverse metric g^ij of the symmetric 3x3 g_ij (the inverse entering the
 * Christoffel definition, Sec. 1; the paper takes it as an input).
 * g: 6 comps in; ginv: 6 comps out. */
tl_status tl_sym_inverse(int64_t n, tl_cfield g, tl_field ginv, void* stream,
                         const tl_tune* tune);

/* Christoffel symbols Gamma^i_jk = 1/2 g^il (d_k g_jl + d_j g_lk - d_l g_jk)
 * (Sec. 1, eq:SpatialChristoffel).  ginv: 6, dg: 18 in; gamma: 18 out. */
tl_status tl_christoffel(int64_t n, tl_cfield ginv, tl_cfield dg, tl_field gamma, void* stream,
                         const tl_tune* tune);

/* Covariant derivative nabla_j beta_i = d_j beta_i - Gamma^k_ij beta_k (Sec. 1,
 * footnote).  gamma: 18, beta: 3, dbeta: 9 in; nabla_beta: 9 out. */
tl_status tl_cov_deriv(int64_t n, tl_cfield gamma, tl_cfield beta, tl_cfield dbeta,
                       tl_field nabla_beta, void* stream, const tl_tune* tune);

/* Metric evolution d_t g_ij = -2 alpha K_ij + nabla_i beta_j + nabla_j beta_i
 * (Sec. 1, eq:dtg_ij).  alpha: 1, K: 6, nabla_beta: 9 in; dtg: 6 out. */
tl_status tl_dtg(int64_t n, tl_cfield alpha, tl_cfield K, tl_cfield nabla_beta, tl_field dtg,
                 void* stream, const tl_tune* tune);

/* ---- Fused chain ---------------------------------------------------------- */

/* d_t g_ij from g, d g, beta, d beta, K and alpha in one pass (Sec. 1,
 * eq:dtg_ij with the covariant derivative of its footnote and
 * eq:SpatialChristoffel substituted): the four steps above with g^ij and
 * Gamma kept in registers (never written to memory),
 * evaluated in the equivalent reduced form
 *   b^l = g^lk beta_k,  F_lij = d_j g_il + d_i g_lj - d_l g_ij,
 *   d_t g_ij = -2 alpha K_ij + d_i beta_j + d_j beta_i - b^l F_lij,
 * which equals the definition because Gamma^k_ij beta_k = 1/2 b^l F_lij.
 * Reads 43 and writes 6 doubles per point. */
tl_status tl_dtg_chain(int64_t n, tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield dbeta,
                       tl_cfield K, tl_cfield alpha, tl_field dtg, void* stream,
                       const tl_tune* tune);

/* Adjoint of tl_dtg_chain (not in the paper: the reverse-mode derivative of the
 * same definitions): given w = dL/d(dtg) (6 comps), writes the gradient
 * of L with respect to every stored input component (an off-diagonal stored
 * slot of g, dg or K receives the sum of its (i,j) and (j,i) partials).
 * g^ij and b^l are recomputed, not stored.  d beta is not an input: d_t g is
 * linear in it, so its gradient depends on w only.  An output whose ptr is
 * NULL is skipped (ld ignored); at least one output must be non-NULL.
 * Reads 40 and writes up to 43 doubles per point. */
tl_status tl_dtg_chain_bwd(int64_t n, tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield K,
                           tl_cfield alpha, tl_cfield w, tl_field g_bar, tl_field dg_bar,
                           tl_field beta_bar, tl_field dbeta_bar, tl_field K_bar,
                           tl_field alpha_bar, void* stream, const tl_tune* tune);

/* tl_dtg_chain and tl_dtg_chain_bwd in one pass, for a cotangent w that is
 * known when the chain is evaluated (a loss linear in d_t g, such as
 * L = sum_s w_s d_t g_s): writes d_t g and the gradients of tl_dtg_chain_bwd
 * (same meaning, layout and order) while reading the shared inputs once --
 * 49 doubles read and up to 49 written per point, against 43 + 6 and 40 + 43
 * for the two calls.  Any output whose ptr is NULL is skipped (ld ignored); at
 * least one must be non-NULL.  Errors as for tl_dtg_chain_bwd. */
tl_status tl_dtg_chain_fwd_bwd(int64_t n, tl_cfield g, tl_cfield dg, tl_cfield beta,
                               tl_cfield dbeta, tl_cfield K, tl_cfield alpha, tl_cfield w,
                               tl_field dtg, tl_field g_bar, tl_field dg_bar, tl_field beta_bar,
                               tl_field dbeta_bar, tl_field K_bar, tl_field alpha_bar,
                               void* stream, const tl_tune* tune);

/* ---- Many subgrids in one launch (multi-domain grids, Sec. 1) ------------- */

/* One subgrid: n points and its seven fields (as for tl_dtg_chain). */
typedef struct {
  int64_t n;
  tl_cfield g, dg, beta, dbeta, K, alpha;
  tl_field dtg;
} tl_domain;

typedef struct tl_batch_plan tl_batch_plan;

/* Builds a plan that evaluates tl_dtg_chain on every domain with one kernel
 * launch over the tiles of all domains, captured once into a HIP graph (by
 * default one block per tile; tune->grid_mult > 0 makes it persistent, each
 * block walking a contiguous chunk of tiles).  The plan copies the domain
 * table and its tile tables to device memory (its only device allocations,
 * freed by tl_batch_plan_destroy) and borrows the domains' buffers, which
 * must outlive it; if any pointer changes, destroy the plan and create a new
 * one.  ndom >= 1; domains with n == 0 are allowed.  Validation is as for
 * tl_dtg_chain, per domain, plus: no domain's output may share an element
 * with any domain's input or output (domains that are point ranges of the
 * same fields are accepted). */
tl_status tl_batch_plan_create(const tl_domain* doms, int32_t ndom, const tl_tune* tune,
                               tl_batch_plan** out);
/* One subgrid of the adjoint: n points, the inputs of tl_dtg_chain_bwd and
 * its gradient outputs (an output whose ptr is NULL is skipped; at least one
 * must be non-NULL when n > 0). */
typedef struct {
  int64_t n;
  tl_cfield g, dg, beta, K, alpha, w;
  tl_field g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar;
} tl_domain_bwd;

/* The same for the adjoint: a plan that evaluates tl_dtg_chain_bwd on every
 * domain with one captured launch.  Ownership, validation and the functions
 * below (launch, info, destroy) are as for tl_batch_plan_create. */
tl_status tl_batch_plan_bwd_create(const tl_domain_bwd* doms, int32_t ndom, const tl_tune* tune,
                                   tl_batch_plan** out);

/* Replays the captured launch on `stream` (asynchronous). */
tl_status tl_batch_plan_launch(tl_batch_plan* plan, void* stream);
/* Launches the same kernel directly, without the graph (asynchronous). */
tl_status tl_batch_plan_launch_direct(tl_batch_plan* plan, void* stream);
/* Total points, tiles and grid size of a plan (any pointer may be NULL). */
tl_status tl_batch_plan_info(const tl_batch_plan* plan, int64_t* points, int64_t* tiles,
                             int64_t* blocks);
/* Waits for all work on the plan's device, then frees the plan (from any
 * current device; the current device is restored); NULL is a no-op. */
tl_status tl_batch_plan_destroy(tl_batch_plan* plan);

/* ---- Many subgrids without allocating ------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): evaluates
 * tl_dtg_chain on every domain with the batched kernel of tl_batch_plan_create
 * -- the same launch, tile order and results as creating a plan with the same
 * doms and tune, calling tl_batch_plan_launch_direct and destroying the plan --
 * but with the plan's tables (domain descriptors, first tile of each domain,
 * tile -> domain map) in a fixed array of device memory that the library
 * holds on each device it runs on, from the first call there until the
 * process ends (about 1.4 MB).  Kernels launched on `stream` write the tables
 * from their kernel arguments, then the batched kernel runs; the call makes no
 * device allocation, no host-to-device copy and no memset, and returns once
 * the launches are queued (asynchronous).  Being kernel launches only, the
 * call may be captured into a HIP graph: each replay writes the tables again
 * before the batched kernel reads them.  The caller passes every input and
 * output, as for a plan; the domains' buffers must stay valid until the work
 * on `stream` has finished.
 * Every call on a device shares that device's array and leaves its tables in
 * it: calls that overlap on one device (on different streams, or from several
 * host threads without ordering between them) race and may read each other's
 * tables; order them on one stream.
 * Limits: 1 <= ndom <= TL_NOALLOC_MAX_DOMAINS, and at most TL_NOALLOC_MAX_TILES
 * tiles in all, a domain of n points taking ceil(n / (block * ppt)) tiles of
 * the resolved launch shape (the default, one block of 128 threads per tile,
 * allows 33.5 M points); beyond either limit TL_ERR_SIZE, before anything is
 * launched.  Validation otherwise as for tl_batch_plan_create. */
#define TL_NOALLOC_MAX_DOMAINS 1024
#define TL_NOALLOC_MAX_TILES 262144
tl_status tl_batch_run_noalloc(const tl_domain* doms, int32_t ndom, const tl_tune* tune,
                               void* stream);

/* ---- The paper's benchmark expressions (Sec. 5.1) ------------------------- */

/* Three-dimensional indices.  A non-symmetric rank-r tensor has 3^r
 * components stored row-major over its indices (A_ij at i*3+j, A_ijk at
 * (i*3+j)*3+k, ...); a mixed B_i^m is stored as B[i*3+m]; K_ij and g_ij are
 * symmetric (s(i,j)); alpha is a scalar field.  in[] holds the right-hand-side
 * tensors in the order they are written; out is the left-hand side.
 *
 *   id                  expression                            in (comps)   out
 *   TL_ASSIGN1          A_i = B_i               eq:Assign1    3            3
 *   TL_ASSIGN2          A_ij = B_ij             eq:Assign2    9            9
 *   TL_ASSIGN3          A_ijk = B_ijk           eq:Assign3    27           27
 *   TL_ADD1             A_i = B_i + C_i         eq:Add1       3 3          3
 *   TL_ADD2             ... + D_i               eq:Add2       3 3 3        3
 *   TL_ADD3             ... + E_i               eq:Add3       3 3 3 3      3
 *   TL_MULT1            A_ij = B_i C_j          eq:Mult1      3 3          9
 *   TL_MULT2            A_ijk = B_i C_j D_k     eq:Mult2      3 3 3        27
 *   TL_MULT3            A_ijkl = B_i C_j D_k E_l eq:Mult3     3 3 3 3      81
 *   TL_CONTRACT1        A_ijkl = B_i^m E_mjkl   eq:Contract1  9 81         81
 *   TL_CONTRACT2        C_j^n B_i^m E_mnkl      eq:Contract2  9 9 81       81
 *   TL_CONTRACT3        D_k^o C_j^n B_i^m E_mnol eq:Contract3 9 9 9 81     81
 *   TL_KIJ              K_ij = 2 alpha g_ij + beta_i beta_j  eq:Kij  1 6 3  6
 *
 * Validation and execution as for the other entry points; a wrong nin or an
 * unknown id returns TL_ERR_INVALID. */
typedef enum {
  TL_ASSIGN1 = 0, TL_ASSIGN2, TL_ASSIGN3, TL_ADD1, TL_ADD2, TL_ADD3, TL_MULT1, TL_MULT2,
  TL_MULT3, TL_CONTRACT1, TL_CONTRACT2, TL_CONTRACT3, TL_KIJ, TL_EXPR_COUNT
} tl_expr_id;

tl_status tl_expr(int32_t expr, int64_t n, const tl_cfield* in, int32_t nin, tl_field out,
                  void* stream, const tl_tune* tune);
/* Number of inputs, their component counts (up to 4) and the output's. */
tl_status tl_expr_shape(int32_t expr, int32_t* nin, int32_t* in_ncomp, int32_t* out_ncomp);

/* ---- Bandwidth reference ---------------------------------------------------- */

/* dst[i] = src[i] for i < n: a plain streaming copy, the library's analogue of
 * a device bandwidth test (Sec. 4, measured bandwidth).  Non-overlapping. */
tl_status tl_bw_copy(int64_t n, const double* src, double* dst, void* stream);

/* Read-only and write-only references: with tl_bw_copy, the measured
 * ceilings of each direction of traffic.  TL_BW_READ reads src[0..n) with
 * 16-byte non-temporal loads; each of its blocks (at most TL_BW_READ_BLOCKS)
 * writes the sum of its share of src to dst[block], so dst must hold
 * TL_BW_READ_BLOCKS doubles, and the sum of those partial sums is the sum of
 * src up to rounding (entries past the number of blocks are not written).
 * TL_BW_WRITE writes dst[i] = 1 for i < n; src is ignored.  Another kind:
 * TL_ERR_INVALID. */
#define TL_BW_READ 1
#define TL_BW_WRITE 2
#define TL_BW_READ_BLOCKS 2048
tl_status tl_bw_stream(int64_t n, int32_t kind, const double* src, double* dst, void* stream);

/* Bandwidth twin of a row's access shape: reads the first nin components of
 * `in` and writes the first nout components of `out` (out_c = sum of the
 * inputs + c) with the library's launch machinery and tuning, and no other
 * arithmetic.  Supported (nin, nout): (1,1), (6,6), (24,18), (30,9), (16,6),
 * (43,6), (40,43) -- the shapes of the rows above; others: TL_ERR_INVALID. */
tl_status tl_bw_twin(int64_t n, int32_t nin, tl_cfield in, int32_t nout, tl_field out,
                     void* stream, const tl_tune* tune);

/* ---- Introspection -------------------------------------------------------------- */

/* Registers and occupancy of one compiled kernel: the counterpart of the
 * paper's table of registers per thread and theoretical occupancy of its
 * generated kernels (Sec. 5.3, tab:registertable). */
typedef struct {
  int32_t block, ppt, flags;   /* the instantiation the tuning resolves to */
  int32_t vgprs;               /* architected vector registers per lane (runtime) */
  int32_t agprs;               /* accumulation vector registers per lane */
  int32_t sgprs;               /* scalar registers per wave, VCC and the other
                                  reserved ones included */
  int32_t scratch_bytes;       /* private (scratch) bytes per lane (runtime) */
  int32_t waves_per_simd;      /* waves of this kernel resident per SIMD when it
                                  is launched with `block` threads per block
                                  (the runtime's occupancy calculator) */
  int32_t max_waves_per_simd;  /* the compiler's bound from registers alone */
  int32_t max_threads;         /* max threads per block for the kernel */
} tl_kernel_attr;

/* Attributes of the kernel that `kernel` ("sym_inverse", "christoffel",
 * "cov_deriv", "dtg", "dtg_chain", "dtg_chain_bwd", "dtg_chain_fwd_bwd",
 * "dtg_chain_batched", "dtg_chain_bwd_batched", or an expression name
 * "assign1" ... "contract3", "kij") would run with `tune` on a large grid
 * (ppt assumes aligned fields).  VGPRs and scratch come from the HIP runtime,
 * SGPRs, AGPRs and the register-bound occupancy from the compiler's resource
 * report, compiled into the library when it was built, waves_per_simd from
 * the runtime's occupancy calculator; a value that cannot be obtained is -1.
 * Needs a HIP device (TL_ERR_HIP otherwise). */
tl_status tl_kernel_info(const char* kernel, const tl_tune* tune, tl_kernel_attr* out);

const char* tl_status_string(tl_status s);
/* Message of the last error on the calling thread ("" if none). */
const char* tl_last_error(void);
int tl_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TL_H */
