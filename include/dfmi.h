/*
 * dfmi.h -- C ABI of the density-fitting contraction library for AMD MI355X (gfx950).
 *
 * The library evaluates the contractions of the packed three-index Cholesky
 * tensor b^P_{mu nu} that density-fitted LASSCF spends its time in
 * (Agarawal et al., arXiv 2505.03755, Sec. "Identification of computational
 * bottlenecks" and "Analysis of computational bottlenecks"):
 *
 *   df_half_transform   Eq. (ao2mo_1), optionally followed by Eq. (ao2mo_2)
 *   df_jk               the "JK call": Eqs. (J_1), (J_2), (K_1), (K_2)
 *   df_active_eri       (uv|wx), the active-space ERIs of the recombination step (Eq. flas)
 *   df_papa             (pu|vw), the g^{p a}_{a a} pattern of the orbital gradient (Eq. MO_conv);
 *                       with DF_PAPA_FULL the (pu|qv) block of Eq. (papa)
 *   df_ppaa             (pq|uv) of Eq. (ppaa), through the AO basis
 *   df_build_cholesky   b^P itself from the three-centre integrals and the metric, Eq. (cholesky)
 *   df_embed_cholesky   b^P in another orbital basis (fragment embedding orbitals)
 *   df_step             all of the above from one shared half transform
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every array argument is a DEVICE pointer (memory of the context's GPU), holding
 *    IEEE float64 values, row major and contiguous.  Sizes are int64_t.
 *  - B is the packed Cholesky tensor, shape [naux][nao*(nao+1)/2], P-major:
 *        B[P*npair + i*(i+1)/2 + j] = b^P_{ij} = b^P_{ji},   i >= j
 *    (the lower-triangular storage of the paper, Sec. "Calculation of effective potentials").
 *  - Densities are passed in factored form, D = C diag(w) C^T, C [nao][nocc].  No spin
 *    factor is applied anywhere: J = J[D] and K = K[D] exactly as in Eqs. (J_1)-(K_2).
 *  - The caller owns every buffer.  Calls that need scratch memory take it from the
 *    workspace attached with df_set_workspace; its size comes from df_workspace_size.
 *    The library never allocates device memory during a call.
 *  - Calls are asynchronous on the context's stream: they return once the work is
 *    enqueued, and every buffer must stay valid until the stream has drained.
 *    Two calls that share one context (and hence one workspace) must not overlap.
 *  - Outputs are overwritten, or, with DF_ACCUMULATE on the calls that take it, added to
 *    (out += result): the sums over P of Eqs. (J_2)-(K_2) and of the ERI blocks can then be
 *    accumulated over blocks of auxiliary rows, as the paper does with its N_blk blocks (Sec.
 *    "Analysis of computational bottlenecks").  Inputs, outputs and the workspace must not
 *    overlap.
 *  - With DF_PREC_SPLIT the bulk products of df_half_transform, df_jk, df_active_eri and df_papa
 *    run in split precision on the int8 matrix cores (see df_split_matmul below) against int8
 *    planes of B registered once per context with df_register_split; df_set_split_slices sets
 *    the slice count.  J-vectors and J stay FP64.
 *  - All arguments are checked before anything is enqueued; on an error return no
 *    output and no workspace byte has been touched, and df_last_error() describes it.
 *  - nocc = 0 or nac = 0 are valid and give zero-sized or zero-valued outputs;
 *    nao >= 1 and naux >= 1 are required.
 */
#ifndef DFMI_H
#define DFMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct df_ctx df_ctx;

typedef enum df_status {
  DF_OK = 0,
  DF_ERR_ARG = -1,          /* null pointer where one is required, overlap, bad context */
  DF_ERR_SHAPE = -2,        /* negative or unsupported size */
  DF_ERR_WORKSPACE = -3,    /* no workspace attached, or smaller than df_workspace_size */
  DF_ERR_HIP = -4,          /* a HIP runtime call failed (message has the HIP error) */
  DF_ERR_UNSUPPORTED = -5   /* unknown flag bit or operation */
} df_status;

/* Operations, for df_workspace_size. */
typedef enum df_op {
  DF_OP_HALF_TRANSFORM = 1,
  DF_OP_JK = 2,
  DF_OP_ACTIVE_ERI = 3,
  DF_OP_PAPA = 4,
  DF_OP_STEP = 5,
  DF_OP_STEP_BACKWARD = 6,
  DF_OP_SPLIT_MATMUL = 7,
  DF_OP_STEP_SPLIT = 8,
  DF_OP_STEP_BACKWARD_SPLIT = 9,
  DF_OP_PPAA = 10,
  DF_OP_BUILD_CHOLESKY = 11,
  DF_OP_EMBED_CHOLESKY = 12
} df_op;

/* Kernel classes reported by df_timing_read. */
typedef enum df_kernel_kind {
  DF_KERNEL_HALF_TRANSFORM = 0,  /* X = b^P C, Eq. (ao2mo_1) */
  DF_KERNEL_JVEC = 1,            /* v_P, Eq. (J_1) */
  DF_KERNEL_COULOMB = 2,         /* J = sum_P v_P b^P, Eq. (J_2) */
  DF_KERNEL_K_SYRK = 3,          /* K tiles, Eqs. (K_1)-(K_2) in factored form */
  DF_KERNEL_K_REDUCE = 4,        /* fixed-order sum of the K split partials */
  DF_KERNEL_MO_TRANSFORM = 5,    /* b^P_{pu} = Cp^T X, Eq. (ao2mo_2) */
  DF_KERNEL_PAPA = 6,            /* (pu|vw) / (pu|qv) contraction over P */
  DF_KERNEL_ERI = 7,             /* (uv|wx) contraction over P */
  DF_KERNEL_OTHER = 8,           /* fills, symmetrisations and coefficient gathers */
  DF_KERNEL_ADJOINT = 9,         /* the products of df_step_backward */
  DF_KERNEL_SPLIT = 10,          /* splitting FP64 operands into int8 slices */
  DF_KERNEL_BUILD = 11,          /* metric Cholesky and forward substitution of df_build_cholesky */
  DF_NUM_KERNEL_KINDS = 12
} df_kernel_kind;

/* Flag bits of calls. */
#define DF_PAPA_FULL 0x1   /* df_papa: return (pu|qv) of Eq. (papa) instead of (pu|vw) */
#define DF_ACCUMULATE 0x2  /* df_half_transform, df_jk, df_active_eri, df_papa: outputs += results */
#define DF_PREC_SPLIT 0x4  /* the same four calls: bulk products in split precision (int8 slices) */

/* Flag bits of df_dims.flags for df_workspace_size only. */
#define DF_CALLER_X  0x10  /* DF_OP_STEP / DF_OP_STEP_BACKWARD / DF_OP_STEP_SPLIT: Xocc, Xact passed in */
#define DF_BWD_GJ    0x20  /* DF_OP_STEP_BACKWARD(_SPLIT): gJ is given */
#define DF_BWD_GK    0x40  /* DF_OP_STEP_BACKWARD(_SPLIT): gK is given */
#define DF_BWD_GERI  0x80  /* DF_OP_STEP_BACKWARD(_SPLIT): geri is given */
#define DF_SPLIT_K_FP64 0x100  /* df_batched_step_split: K in FP64 from the split-precision X_occ */
#define DF_WEIGHTED  0x200  /* DF_OP_JK with DF_PREC_SPLIT: weights w are given (their K operand is split too) */

/* Problem sizes for df_workspace_size; fields an operation does not use are ignored. */
typedef struct df_dims {
  int64_t naux, nao;
  int64_t ndm;    /* number of densities in a JK call (>= 1) */
  int64_t nocc;   /* columns of each density factor */
  int64_t nac;    /* active orbitals */
  int64_t np;     /* columns of Cp (MO space p) */
  int64_t nq;     /* columns of Cq (DF_PAPA_FULL, DF_OP_PPAA) */
  int64_t ncol;   /* columns of C in df_half_transform; nemb for DF_OP_EMBED_CHOLESKY */
  int64_t n2;     /* columns of C2 in df_half_transform (0 if no second transform) */
  int flags;
  int nslice;     /* int8 slices per operand (split-precision ops) */
  int64_t m, n, k;  /* product sizes of DF_OP_SPLIT_MATMUL */
} df_dims;

/* Create a context on HIP device `device` that enqueues onto `stream`
 * (a hipStream_t; NULL means the null stream).  *ctx is set on success.  No HIP call is
 * made here: the device is selected by the first call that enqueues work, and an invalid
 * device is reported there as DF_ERR_HIP. */
df_status df_create(df_ctx** ctx, int device, void* stream);

/* Destroy a context (NULL is allowed).  Does not free the attached workspace. */
df_status df_destroy(df_ctx* ctx);

/* Message of the last error on this context ("" if none).  The string is owned by the
 * context and valid until its next call.  With ctx == NULL: the last df_create error. */
const char* df_last_error(const df_ctx* ctx);

/* Change the stream later calls enqueue onto. */
df_status df_set_stream(df_ctx* ctx, void* stream);

/* Attach caller-owned device memory of `bytes` bytes as the workspace (NULL, 0 detaches).
 * ptr must be 256-byte aligned (DF_ERR_ARG otherwise); 4096-byte alignment keeps the int8
 * planes of the split-precision calls, placed on 4 KB offsets, in whole 1 KB blocks per page. */
df_status df_set_workspace(df_ctx* ctx, void* ptr, size_t bytes);

/* Per-kernel timing.  While enabled, every launch the context makes is bracketed by two HIP
 * events recorded on the context's stream (so each interval is that kernel's duration).
 * df_timing_read waits for the recorded events, writes the summed milliseconds and launch
 * counts per df_kernel_kind into ms[0..n) and launches[0..n) (kinds >= n are dropped), and
 * starts a new interval.  Timing adds two event records per launch; leave it off otherwise. */
df_status df_set_timing(df_ctx* ctx, int enable);
df_status df_timing_read(df_ctx* ctx, double* ms, int64_t* launches, int n);

/* Bytes of workspace that operation `op` needs for the sizes in *dims, with no scratch limit.
 * dims->flags carries the call's flags (DF_PAPA_FULL, DF_ACCUMULATE, DF_PREC_SPLIT with
 * dims->nslice slices) and the DF_CALLER_X / DF_BWD_* bits below. */
df_status df_workspace_size(df_op op, const df_dims* dims, size_t* bytes);

/* The same for calls made on `ctx`: its scratch limit (df_set_scratch_limit) applies to
 * DF_OP_STEP_BACKWARD, and with DF_PREC_SPLIT a dims->nslice of 0 stands for the context's slice
 * count.  DF_ERR_WORKSPACE when the scratch limit is below the smallest workspace the operation
 * can run in (one auxiliary row per chunk). */
df_status df_workspace_query(df_ctx* ctx, df_op op, const df_dims* dims, size_t* bytes);

/* Bound on the workspace of df_step_backward, in bytes (0: no bound, the default).  With a bound
 * the adjoint runs over the auxiliary index in chunks of rows: per chunk it forms (or, when the
 * caller passes them, reads) the half transforms of those rows and the products that need them,
 * and it accumulates the chunk's part of dCocc and dCact in a fixed order.  So the
 * half-transformed tensor is recomputed chunk by chunk rather than stored whole when it does not
 * fit (Sec. "Analysis of computational bottlenecks": blocking along P bounds the peak memory).
 * The chunk is the most rows whose workspace stays within the bound; df_backward_chunk reports
 * it.  Results agree with the unbounded call up to FP64 rounding order. */
df_status df_set_scratch_limit(df_ctx* ctx, size_t bytes);

/* Rows of the auxiliary index per chunk that df_step_backward on `ctx` uses for these sizes
 * (dims as for DF_OP_STEP_BACKWARD); *rows = naux without a bound.  DF_ERR_WORKSPACE as in
 * df_workspace_query. */
df_status df_backward_chunk(df_ctx* ctx, const df_dims* dims, int64_t* rows);

/* Slice count of DF_PREC_SPLIT calls on this context (in [4, 8], default 7). */
df_status df_set_split_slices(df_ctx* ctx, int nslice);

/* Registers the int8 planes Bs and exponents Be that df_split_cholesky made from B (with
 * `nslice` slices) for DF_PREC_SPLIT calls on this context.  A call with DF_PREC_SPLIT uses the
 * registration whose B pointer, naux and nao equal its own and whose nslice is the context's
 * slice count; without one it fails with DF_ERR_ARG.  Registering the same (B, naux, nao,
 * nslice) again replaces the planes; Bs = NULL removes that registration.  The buffers stay
 * caller-owned and must stay valid while registered.  At most 16 registrations. */
df_status df_register_split(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const int8_t* Bs,
                            const int* Be, int nslice);

/*
 * Half transform, Eq. (ao2mo_1):       X[P][mu][c] = sum_nu b^P_{mu nu} C[nu][c]
 * and optionally Eq. (ao2mo_2):        Y[P][p][c]  = sum_mu C2[mu][p] X[P][mu][c]
 *
 *   B  [naux][npair]      packed Cholesky vectors (input)
 *   C  [nao][ncol]        coefficients (input), ncol >= 1
 *   X  [naux][nao][ncol]  output; the untransformed AO index comes first, as in b^P_{e2 p1}
 *   C2 [nao][n2], Y [naux][n2][ncol]  both NULL (n2 = 0) or both given
 * flags: DF_ACCUMULATE (X += b^P C, Y += C2^T (b^P C)), DF_PREC_SPLIT (both products from int8
 *   slices: rows (P, mu) of b^P against rows c of C; rows p of C2 against rows (P, c) of X).
 * Workspace: df_workspace_size(DF_OP_HALF_TRANSFORM, {naux, nao, ncol, n2, flags, nslice})
 * (a zero-padded copy of C; with both flags set and C2, also the new X before it is added).
 */
df_status df_half_transform(df_ctx* ctx, const double* B, int64_t naux, int64_t nao,
                            const double* C, int64_t ncol, double* X,
                            const double* C2, int64_t n2, double* Y, int flags);

/*
 * JK call for ndm densities D_k = C_k diag(w_k) C_k^T (Eqs. J_1, J_2, K_1, K_2):
 *   v[k][P] = sum_{ij} b^P_{ij} (D_k)_{ij}
 *   J[k]    = sum_P v[k][P] b^P
 *   K[k]    = sum_P (b^P C_k) diag(w_k) (b^P C_k)^T      (= sum_P b^P D_k b^P)
 *
 *   Cocc [ndm][nao][nocc]  density factors (input)
 *   w    [ndm][nocc]       signed occupation weights, or NULL for all ones
 *   J, K [ndm][nao][nao]   outputs (symmetric, both triangles written); either may be NULL
 *   v    [ndm][naux]       output, or NULL
 * flags: DF_ACCUMULATE (J, K, v += the results); DF_PREC_SPLIT (X_k = b^P C_k and every K_k from
 *   int8 slices; v and J in FP64 from that X).
 * Workspace: df_workspace_size(DF_OP_JK, {naux, nao, ndm, nocc, flags, nslice}).
 */
df_status df_jk(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int64_t ndm,
                const double* Cocc, int64_t nocc, const double* w,
                double* J, double* K, double* v, int flags);

/*
 * df_jk without any allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and checks as df_jk in FP64; flags: DF_ACCUMULATE only (DF_PREC_SPLIT is DF_ERR_UNSUPPORTED).
 * No workspace is attached or used: the scratch is one 128 MiB device array inside the library
 * (one copy per GPU, held until the process ends; its address is looked up once per device on the
 * first call there).  The auxiliary rows run in blocks whose workspace fits it (J and K add up
 * over the blocks, so the sums are ordered differently from df_jk's: equal to rounding);
 * DF_ERR_WORKSPACE when a single auxiliary row does not fit (about ndm (nao^2 + 2 nao nocc) doubles
 * must stay below 128 MiB).
 * Every call on one GPU shares that array, and it keeps the last call's contents: calls that may
 * overlap on one GPU (two streams, two contexts, two threads) race and must be serialised by the
 * caller.  Calls no hipMalloc, hipFree or other allocating routine, and records no timing events.
 */
df_status df_jk_noalloc(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int64_t ndm,
                        const double* Cocc, int64_t nocc, const double* w,
                        double* J, double* K, double* v, int flags);

/*
 * Active-space ERIs:  b_uv[P][u][v] = (Cact^T b^P Cact)_{uv},
 *                     eri[u][v][w][x] = sum_P b_uv[P][u][v] b_uv[P][w][x]
 *   Cact [nao][nac] (input); eri [nac]^4 (output); buv [naux][nac][nac] (output or NULL)
 * flags: DF_ACCUMULATE (eri, buv += the results); DF_PREC_SPLIT (b^P Cact, b_uv and eri from int8
 *   slices).
 * Workspace: df_workspace_size(DF_OP_ACTIVE_ERI, {naux, nao, nac, flags, nslice}).
 */
df_status df_active_eri(df_ctx* ctx, const double* B, int64_t naux, int64_t nao,
                        const double* Cact, int64_t nac, double* eri, double* buv, int flags);

/*
 * papa block.  b_pu[P] = Cp^T b^P Cact, b_vw[P] = Cact^T b^P Cact.
 *   default:       out[p][u][v][w] = (pu|vw) = sum_P b_pu[P][p][u] b_vw[P][v][w]
 *                  (Cq must be NULL, nq = 0);  out is [np][nac][nac][nac]
 *   DF_PAPA_FULL:  out[p][u][q][v] = (pu|qv) = sum_P b_pu[P][p][u] b_qv[P][q][v]   (Eq. papa)
 *                  with b_qv[P] = Cq^T b^P Cact;  out is [np][nac][nq][nac]
 *   Cp [nao][np], Cact [nao][nac], Cq [nao][nq] (inputs)
 * flags: DF_PAPA_FULL (above), DF_ACCUMULATE (out += the result), DF_PREC_SPLIT (b^P Cact, the
 *   second transforms and the contraction over P from int8 slices).
 * Workspace: df_workspace_size(DF_OP_PAPA, {naux, nao, nac, np, nq, flags, nslice}).
 */
df_status df_papa(df_ctx* ctx, const double* B, int64_t naux, int64_t nao,
                  const double* Cp, int64_t np, const double* Cact, int64_t nac,
                  const double* Cq, int64_t nq, double* out, int flags);

/*
 * ppaa block of Eq. (ppaa):  (pq|uv) = sum_P b^P_pq b^P_uv  with  b^P_pq = (Cp^T b^P Cq)_{pq},
 * b^P_uv = (Cact^T b^P Cact)_{uv}.
 *   out[pair(u,v)][p][q] = (pq|uv),  pair(u,v) = u(u+1)/2 + v for u >= v (the (uv) index packed
 *   like B, since (pq|uv) = (pq|vu));  out is [nac(nac+1)/2][np][nq]
 *   Cp [nao][np], Cq [nao][nq], Cact [nao][nac] (inputs).  Cq = NULL (with nq = 0) means Cq = Cp.
 * Evaluated through the AO basis: W_uv = sum_P b^P_uv b^P over the packed pairs (one product with
 * B per chunk of uv pairs), then out[uv] = Cp^T W_uv Cq, so b^P_pq is never formed.  That costs
 * 2 N_aux npair N_uv + 2 N_uv N_ao nq (N_ao + np) FLOP against 2 N_aux N_ao nq (N_ao + np) +
 * 2 N_aux np nq N_uv for the MO route (N_uv = nac(nac+1)/2), far less when N_uv < N_aux.
 * The uv pairs run in chunks that keep the per-chunk buffers near 2 GiB (B is read once per chunk).
 * Errors: DF_ERR_ARG for a missing Cp/Cact/out (when the output is not empty), nq != 0 without
 * Cq, or overlapping buffers; DF_ERR_SHAPE for negative sizes; DF_ERR_UNSUPPORTED for flags != 0.
 * Workspace: df_workspace_size(DF_OP_PPAA, {naux, nao, nac, np, nq}) (nq = 0: nq = np).
 */
df_status df_ppaa(df_ctx* ctx, const double* B, int64_t naux, int64_t nao,
                  const double* Cp, int64_t np, const double* Cq, int64_t nq,
                  const double* Cact, int64_t nac, double* out, int flags);

/*
 * Cholesky vectors from the three-centre integrals, Eq. (cholesky):
 *   (mu nu|lam sig) ~ (mu nu|P) (P|Q)^-1 (Q|lam sig) = sum_P b^P_{mu nu} b^P_{lam sig}
 * with (P|Q) = L L^T and B = L^-1 E, E[Q][pair] = (Q|mu nu) packed like B.
 *   metric [naux][naux]: (P|Q), symmetric positive definite; its lower triangle is read.
 *   eri3 [naux][npair]: (Q|mu nu).
 *   L [naux][naux] (output): the Cholesky factor, lower triangular, upper part zeroed.
 *       L may be `metric` itself (factored in place).
 *   B [naux][npair] (output): the Cholesky vectors.  B may be `eri3` itself (in place).
 *   info: one device int, written 0 on success, else P + 1 for the first auxiliary index P
 *       whose pivot is not positive (the metric is not positive definite to working
 *       precision); L and B are then undefined.  It is written on the stream, so read it after
 *       the stream has drained.
 * The factorisation runs in 128-wide block columns, right-looking: each diagonal block is
 * factored and inverted by one workgroup, the panel below is multiplied by the inverted block,
 * and the trailing matrix takes the panel's update as one product.  The metric's strictly upper
 * part, when factored in place, is overwritten (zeroed at the end).  The substitution runs in block rows,
 * B_k = L_kk^-1 (E_k - L_{k,<k} B_{<k}), the update as one product over all earlier rows.
 * Requires 128 * npair < 2^32 and naux^2 < 2^32 (DF_ERR_SHAPE otherwise).
 * Errors: DF_ERR_ARG for NULL pointers or overlapping buffers other than the two in-place
 * pairs; DF_ERR_SHAPE for sizes; DF_ERR_UNSUPPORTED for flags != 0.
 * Workspace: df_workspace_size(DF_OP_BUILD_CHOLESKY, {naux, nao}).
 */
df_status df_build_cholesky(df_ctx* ctx, const double* metric, const double* eri3, int64_t naux, int64_t nao,
                            double* L, double* B, int* info, int flags);

/*
 * Cholesky vectors in another orbital basis, e.g. a fragment's embedding orbitals (effective
 * potentials are built the same way in the AO and in the embedding basis, Sec. "Calculation of
 * effective potentials"):
 *   Be[P][pair(e, f)] = (M^T b^P M)_{ef},  M [nao][nemb] (input),  Be [naux][nemb(nemb+1)/2]
 * packed like B.  P runs in chunks that keep b^P M and M^T b^P M near 1 GiB.
 * Errors: DF_ERR_ARG for missing M/Be (nemb > 0) or overlaps; DF_ERR_SHAPE for sizes;
 * DF_ERR_UNSUPPORTED for flags != 0.
 * Workspace: df_workspace_size(DF_OP_EMBED_CHOLESKY, {naux, nao, ncol = nemb}).
 */
df_status df_embed_cholesky(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* M, int64_t nemb,
                            double* Be, int flags);

/*
 * One forward pass of the whole path from a single half transform X = b^P [Cocc | Cact]:
 * J, K and v of D = Cocc diag(w) Cocc^T (as df_jk with ndm = 1), eri = (uv|wx) and
 * papa = (pu|vw) (as df_active_eri and df_papa).  Any of J, K, v, eri, papa may be NULL.
 *   Xocc [naux][nao][nocc], Xact [nao][naux][nac]: optional outputs (both or neither; one of
 *   zero size may be NULL) that
 *   receive the half-transformed factors b^P Cocc (P-major) and b^P Cact (AO-major), e.g. to be
 *   handed to df_step_backward; when given they replace the workspace's copies.
 * Workspace: df_workspace_size(DF_OP_STEP, {naux, nao, 1, nocc, nac, np,
 *            flags = DF_CALLER_X if Xocc/Xact are given}).
 */
df_status df_step(df_ctx* ctx, const double* B, int64_t naux, int64_t nao,
                  const double* Cocc, int64_t nocc, const double* w,
                  const double* Cact, int64_t nac, const double* Cp, int64_t np,
                  double* J, double* K, double* v, double* eri, double* papa,
                  double* Xocc, double* Xact, int flags);

/*
 * Vector-Jacobian product of df_step's (J, K, eri) as functions of (Cocc, Cact), unit
 * weights (the adjoint used for the orbital-rotation gradient of the differentiable step):
 *   dCocc = 2 M Cocc + sum_P b^P S b^P Cocc,   M = sum_P <b^P, gJ> b^P,   S = gK + gK^T
 *   dCact = sum_P (b^P Cact)(Z_P + Z_P^T),      Z_P[u][v] = sum_wx (geri[uvwx] + geri[wxuv]) b^P_wx
 *   gJ, gK [nao][nao], geri [nac]^4: cotangents, each may be NULL (= zero)
 *   Xocc, Xact: the half transforms from df_step (both or neither; one of zero size may be
 *            NULL); both NULL recomputes them
 *   dCocc [nao][nocc], dCact [nao][nac]: outputs (overwritten)
 * With a scratch limit on the context (df_set_scratch_limit) the auxiliary rows run in chunks,
 * each chunk's half transforms recomputed (or read from Xocc, Xact) into bounded workspace.
 * Workspace: df_workspace_query(ctx, DF_OP_STEP_BACKWARD, {naux, nao, 1, nocc, nac,
 *            flags = DF_BWD_GJ|DF_BWD_GK|DF_BWD_GERI for the given cotangents, | DF_CALLER_X}).
 */
df_status df_step_backward(df_ctx* ctx, const double* B, int64_t naux, int64_t nao,
                           const double* Cocc, int64_t nocc, const double* Cact, int64_t nac,
                           const double* gJ, const double* gK, const double* geri,
                           const double* Xocc, const double* Xact,
                           double* dCocc, double* dCact, int flags);

/*
 * Batched fragment subproblems (the embedding-space problems of the fragment CASSCFs, Sec.
 * "Calculation of effective potentials"): problem i has its own packed B, N_ao, N_aux and ndm
 * densities D_k = C_k C_k^T (unit weights), and asks for
 *   J[k], K[k] as in df_jk, (uv|wx) as in df_active_eri, the full (pu|qv) of Eq. (papa)
 *   with p, q over the columns of Cp (as df_papa with DF_PAPA_FULL and Cq = Cp), and (pq|uv)
 *   of Eq. (ppaa) over the same p, q (as df_ppaa with Cq = Cp).
 * The half transforms of all problems ([C_1 .. C_ndm | Cact] against b^P) run as one grouped
 * launch, and so do the K tiles; problems are ordered largest first inside each launch.
 * (pq|uv) runs last, problem after problem, through one workspace region sized for the largest.
 * Any output may be NULL.  Inputs and outputs of all problems must not overlap each other.
 */
typedef struct df_problem {
  const double* B;      /* [naux][npair] packed Cholesky vectors */
  int64_t naux, nao;
  int64_t ndm;          /* densities (>= 1) */
  const double* Cocc;   /* [ndm][nao][nocc] */
  int64_t nocc;
  const double* Cact;   /* [nao][nac] */
  int64_t nac;
  const double* Cp;     /* [nao][np] */
  int64_t np;
  double* J;            /* [ndm][nao][nao] */
  double* K;            /* [ndm][nao][nao] */
  double* eri;          /* [nac][nac][nac][nac] */
  double* papa;         /* [np][nac][np][nac] */
  double* ppaa;         /* [nac(nac+1)/2][np][np], the (uv) index packed as in df_ppaa */
} df_problem;

/* Workspace bytes for df_batched_step on these problems. */
df_status df_batched_workspace_size(const df_problem* probs, int nprob, size_t* bytes);
df_status df_batched_step(df_ctx* ctx, const df_problem* probs, int nprob, int flags);

/*
 * Autotuning of df_batched_step's grouped launches (tile shapes chosen by measurement rather
 * than by a fixed rule).  With enable != 0, the first df_batched_step on a problem group whose
 * shape the context has not seen runs every candidate of each phase twice on the call's own
 * buffers, timed with events on the context's stream.  The phases are the half-transform
 * tile (176, 96, 48: the column width on one row of waves; 128: 128 x 128 tiles on 2 x 2 waves,
 * with each problem's rows past its last whole 128-row band on 64 x 176 tiles where that pads
 * less) and the K tile (64, 128) with its split target (16, 4, 64 rounds of resident
 * workgroups).  The call keeps the fastest of each phase in the context's table, keyed
 * by every problem's (naux, nao, ndm, nocc, nac, np) and its requested outputs, then computes
 * its outputs with them.
 *   - Such a call waits for the GPU.  It is never made while the stream is being captured;
 *     under capture the defaults (or a stored choice) are used.
 *   - Later calls with the same shape use the stored choice, whether tuning is on or off.
 *   - Results do not depend on the choice beyond FP64 rounding order.
 *   - df_batched_workspace_size covers every candidate.
 * df_batched_tuning reports the configuration df_batched_step would use for a group: the
 * stored one (*tuned = 1) or the defaults (*tuned = 0).  df_batched_set_tuning stores a choice
 * for a group's shape (each value from the candidate lists above, else DF_ERR_ARG), e.g. to
 * replay a measured configuration.  None of these calls allocates device memory.
 */
df_status df_set_autotune(df_ctx* ctx, int enable);
df_status df_batched_tuning(df_ctx* ctx, const df_problem* probs, int nprob, int* half_tile_n, int* k_tile,
                            int* k_rounds, int* tuned);
df_status df_batched_set_tuning(df_ctx* ctx, const df_problem* probs, int nprob, int half_tile_n, int k_tile,
                                int k_rounds);

/*
 * The tuning table outlives the context in a file (JSON, format "dfmi-autotune/1"): one entry per
 * problem-group shape with its operation ("df_batched_step"), precision ("fp64"), the device's gfx
 * architecture ("gfx950"; empty for choices set with df_batched_set_tuning, which hold on any
 * device) and the chosen half-transform tile, K tile and K split target.
 *   df_autotune_save writes the context's whole table to path (a temporary file renamed into
 *     place); DF_ERR_ARG if it cannot be written.
 *   df_autotune_load merges the entries of path into the table (file entries replace stored ones
 *     of the same architecture and shape; entries of other operations or precisions, or with a
 *     configuration outside the candidate lists, are skipped); DF_ERR_ARG if the file cannot be
 *     read or is not in this format.  Entries of another architecture stay unused.
 * With the environment variable DFMI_AUTOTUNE_CACHE naming a file, df_create loads it when it
 * exists (a file in another format fails df_create), and every df_batched_step that tunes merges
 * the file's current entries and rewrites it with its new choice.  Neither call touches the GPU;
 * df_batched_tuning, df_batched_set_tuning and df_batched_step ask the runtime for the device's
 * architecture once per context (without a device only architecture-free entries apply).
 */
df_status df_autotune_save(df_ctx* ctx, const char* path);
df_status df_autotune_load(df_ctx* ctx, const char* path);

/*
 * df_batched_step in split precision: the same outputs of the same problems, with the half
 * transform, every density's K, the second transforms, (uv|wx) and the full (pu|qv) as int8
 * slice products (nslice slices, as in df_step_split); J and the J-vectors stay FP64.
 *   - Bs[i], Be[i] are problem i's planes and exponents from df_split_cholesky with the same
 *     nslice.
 *   - Problems run one after another in the given order and share one workspace region,
 *     df_batched_split_workspace_size(probs, nprob, nslice) bytes (the largest problem's need).
 *   - The K products of all densities of a problem run as one launch.
 *   - flags = DF_SPLIT_K_FP64 computes K in FP64 from X_occ (the exchange product of
 *     df_batched_step) instead of splitting every density's X_occ, which for many densities
 *     costs more than the int8 product saves.  The workspace query takes the same flags.
 *   - (pq|uv) is computed in FP64, as in df_batched_step, after the problem's other outputs.
 */
df_status df_batched_split_workspace_size(const df_problem* probs, int nprob, int nslice, int flags, size_t* bytes);
df_status df_batched_step_split(df_ctx* ctx, const df_problem* probs, const int8_t* const* Bs, const int* const* Be,
                                int nprob, int nslice, int flags);

/*
 * Split precision on the int8 matrix cores.  An FP64 row x is cut into nslice int8 slices,
 *   x[k] ~= 2^e sum_{s < nslice} a_s[k] 2^-(6 + 7 s),   a_s in [-64, 64],  max|x| < 2^e,
 * exactly up to a residual below 2^(e - 7 nslice); a product keeps the slice pairs with
 * s + t < nslice, summed exactly in int32 and then in FP64.  For two rows of length K the
 * error is below K (nslice + 4) 2^(e_a + e_b - 7 nslice) plus FP64 rounding; nslice = 7 gives
 * FP64-level results.  nslice must be in [4, 8].  This is the mixed-precision direction the
 * paper lists as future work (Sec. Conclusions), applied to Eqs. (ao2mo_1), (K_2), (ao2mo_2)
 * and (papa).
 */

/*
 * C[m][n] = sum_k A[m][k] B[n][k] by the split method.
 *   A [M][lda], B [N][ldb] (lda, ldb >= K), C [M][ldc] (ldc >= N), row major, FP64, device.
 * Workspace: df_workspace_size(DF_OP_SPLIT_MATMUL, {m = M, n = N, k = K, nslice}).
 */
df_status df_split_matmul(df_ctx* ctx, const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb,
                          int64_t N, int64_t K, int nslice, double* C, int64_t ldc, int flags);

/*
 * One-time split of the Cholesky vectors for df_step_split: the rows (P, mu) of the unpacked
 * b^P (Eq. cholesky) as int8 planes.
 *   Bs: nslice * R * kpad64(nao) int8 (R = naux * nao rounded up to a multiple of 32, kpad64(n) =
 *   n rounded up to a multiple of 64) in 1 KB blocks of 32 rows x 32 k: block (s, g, b) of slice
 *   s, row group g, k block b at byte ((s * R / 32 + g) * kpad64(nao) / 32 + b) * 1024, its
 *   16-byte slot rr + 32 c holding k = 32 b + 16 c + [0, 16) of row 32 g + rr; zeros past the
 *   last row and past nao.  Row r = P * nao + mu is b^P_{mu, k} over k.
 *   Be [naux * nao] int32 exponents; both caller-owned device buffers, overwritten; Bs 16-byte
 *   aligned (DF_ERR_ARG otherwise; 1 KB alignment, no block across a page, reads fastest).
 *   naux * nao <= 2^31 - 32.  No workspace.
 */
df_status df_split_cholesky(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int nslice, int8_t* Bs,
                            int* Be, int flags);

/*
 * The same split for products that contract over (P, nu): the rows mu of the DF tensor over
 * k = P * nao + nu (element b^P_{mu nu}), for df_step_backward_split.
 *   Bt: nslice * rpad32(nao) * kpad64(naux * nao) int8 in the block layout of Bs (rows mu),
 *   Bte [nao] int32 exponents (of max over P and nu of |b^P_{mu nu}|); caller-owned device
 *   buffers, overwritten; Bt 16-byte aligned (1 KB reads fastest).  naux * nao <= 2^30.  No workspace.
 */
df_status df_split_cholesky_t(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int nslice, int8_t* Bt,
                              int* Bte, int flags);

/*
 * df_step in split precision (unit weights): the half transform (against Bs, Be from
 * df_split_cholesky with the same nslice), K, the second transforms, (uv|wx) and (pu|vw) are
 * split products; the J-vector v and J (from the packed B) are FP64.  Outputs as in df_step;
 * any of J, K, v, eri, papa may be NULL.  Xocc [naux][nao][nocc] and Xact [nao][naux][nac]
 * (the layouts of df_step), both or neither, receive the half-transformed factors for
 * df_step_backward_split (NULL only for an empty one).
 * Workspace: df_workspace_size(DF_OP_STEP_SPLIT, {naux, nao, 1, nocc, nac, np, nslice,
 *            flags = DF_CALLER_X if Xocc/Xact are given}).
 */
df_status df_step_split(df_ctx* ctx, const double* B, const int8_t* Bs, const int* Be, int nslice, int64_t naux,
                        int64_t nao, const double* Cocc, int64_t nocc, const double* Cact, int64_t nac,
                        const double* Cp, int64_t np, double* J, double* K, double* v, double* eri, double* papa,
                        double* Xocc, double* Xact, int flags);

/*
 * df_step_backward in split precision: in the exchange part, Y_P = S X_P (S = gK + gK^T) in
 * FP64 and sum_P b^P Y_P as a slice product against Bt, Bte (df_split_cholesky_t, same nslice).
 * The Coulomb part (2 M Cocc) and the active-space part stay FP64, as in df_step_backward.
 * Xocc is required with gK and Xact with geri; there is no recomputation here.  Arguments,
 * outputs and cotangent rules are otherwise as in df_step_backward; nao <= 32768.
 * Workspace: df_workspace_size(DF_OP_STEP_BACKWARD_SPLIT, {naux, nao, 1, nocc, nac, nslice,
 *            flags = DF_BWD_GJ | DF_BWD_GK | DF_BWD_GERI for the given cotangents}).
 */
df_status df_step_backward_split(df_ctx* ctx, const double* B, const int8_t* Bt, const int* Bte, int nslice,
                                 int64_t naux, int64_t nao, const double* Cocc, int64_t nocc, const double* Cact,
                                 int64_t nac, const double* gJ, const double* gK, const double* geri,
                                 const double* Xocc, const double* Xact, double* dCocc, double* dCact, int flags);

#ifdef __cplusplus
}
#endif

#endif /* DFMI_H */
