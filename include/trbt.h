/*
 * trbt.h -- tridiagonal-to-banded eigenvector back-transformation on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation (Yu et al., "GPU-Acceleration of the ELPA2 Distributed
 * Eigensolver for Dense Symmetric and Hermitian Eigenproblems", Sec. 2.2.2,
 * Eq. 2stage_bkwd1 and Eq. kernel):
 *
 *     Y = Q^* X,   Q^* = H_0 H_1 ... H_{K-1},   H_k = I - tau_k v_k v_k^H,
 *
 * i.e. every Householder reflector produced by the banded-to-tridiagonal
 * bulge chasing (Sec. 2.2.1, Eq. householder) is applied to every column of
 * the eigenvector matrix in exactly the reverse of its generation order:
 *
 *     for k = K-1 down to 0:   z[r0_k : r0_k+len_k] -= tau_k v_k (v_k^H z[...])
 *
 * Reflector geometry (0-based; the paper's stage i = s+1, sweep j+1):
 *   stages s = 0 .. n-3; stage s has S_s = ceil((n-s-2)/nbw) sweeps (slots)
 *   (none when nbw = 1, where the band is already tridiagonal);
 *   reflector (s, j) acts on rows [r0, r0+len) with r0 = s+1+j*nbw,
 *   len = min(nbw, n-r0) >= 2; generation order is stage-major, slot-minor,
 *   so reflector (s, j) has index k = S_0 + ... + S_{s-1} + j.
 *
 * Data layout:
 *   hh_v    K x nbw, reflector-contiguous (reflector k at hh_v + k*nbw), in
 *           generation order.  v[0] is read, not assumed to be 1.  Entries
 *           at positions >= len_k are ignored.
 *   hh_tau  K scalars.
 *   Z       n x nev, column-major (LAPACK/ELPA convention), leading
 *           dimension ldz >= max(1, n).  Overwritten in place with Y.
 *           Rows n .. ldz-1 are never read or written.
 *
 * All data pointers are DEVICE pointers.  The caller owns every buffer.
 * Calls are asynchronous on the given HIP stream (pass the hipStream_t as
 * void*; NULL means the default stream) and reentrant.  The only state the
 * library keeps between calls is a per-device cache of the architecture
 * check (filled on a device's first call, never invalidated) and the plans
 * a caller creates.  No entry point below allocates device memory or
 * synchronizes the device, except plan creation and destruction and
 * trbt_work_check.  Kernel-time faults surface at the caller's next
 * synchronization, not as a return code; the bounded inter-workgroup waits
 * of the blocked kernels report a timeout through the workspace's fault
 * word (trbt_work_check).
 *
 * Return codes: TRBT_SUCCESS (0); -i when argument i (1-based) is invalid,
 * checked on the host before anything is launched; or one of the
 * TRBT_ERR_* codes below.  No C++ exception crosses this interface.
 */
#ifndef TRBT_H
#define TRBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRBT_SUCCESS 0
#define TRBT_ERR_DEVICE (-100)    /* current device is not gfx950          */
#define TRBT_ERR_WORKSPACE (-101) /* work too small or misaligned          */
#define TRBT_ERR_HIP (-102)       /* a HIP runtime call / launch failed    */
#define TRBT_ERR_INTERNAL (-103)  /* unexpected state (should not happen)  */
#define TRBT_ERR_SCRATCH (-104)   /* problem too large for the fixed scratch
                                     of an allocation-free entry point     */

#define TRBT_NBW_MAX 256          /* largest semi-bandwidth accepted       */
#define TRBT_WORK_ALIGN 256       /* required alignment of `work`, bytes   */

/* Complex FP64 element: layout-compatible with hipDoubleComplex and with
 * torch.complex128 / numpy complex128. */
typedef struct {
    double re, im;
} trbt_z;

/* Host-only helpers, pure functions (no HIP calls).
 * trbt_num_reflectors: K for (n, nbw); 0 when n < 3 or nbw == 1.
 * trbt_stage_offsets:  off[s] = generation index of reflector (s, 0) for
 *                      s = 0..n-2 (off[n-2] = K); needs n >= 2.
 * Errors: -1 (n < 0), -2 (nbw outside [1, TRBT_NBW_MAX]), -3 (null out). */
int trbt_num_reflectors(int64_t n, int nbw, int64_t *K);
int trbt_stage_offsets(int64_t n, int nbw, int64_t *off);

/* Bytes of device workspace the back-transformation of (n, nbw, nev) needs
 * (real: is_complex = 0, complex: 1).  The workspace holds the per-block
 * compact-WY factors the blocked kernels precompute (nbw a multiple of 16
 * up to 128); it is 0 for shapes served by the unblocked kernel.  The same workspace can be reused by any
 * later call with the same or smaller sizes.  Errors as for the transform
 * (-1 n, -2 nbw, -3 nev; -4 null `bytes`). */
int trbt_workspace_bytes(int64_t n, int nbw, int64_t nev, int is_complex, size_t *bytes);

/* Y = Q^* X in place (Eq. 2stage_bkwd1), real FP64.
 * Arguments: 1 n >= 0, 2 nbw in [1, TRBT_NBW_MAX], 3 0 <= nev <= n,
 * 4 hh_v, 5 hh_tau (non-null unless K == 0 or nev == 0), 6 Z (non-null
 * unless nev == 0 or n == 0), 7 ldz >= max(1, n), 8 work (device, aligned
 * to TRBT_WORK_ALIGN; may be NULL when 9 work_bytes is 0 and
 * trbt_workspace_bytes reports 0), 9 work_bytes, 10 stream.
 * The contents of `work` on entry do not matter; on exit it holds the
 * fault word (read it with trbt_work_check: nonzero means Z is invalid)
 * and otherwise unspecified data.  n < 3, nbw == 1 or nev == 0 return TRBT_SUCCESS without
 * touching Z. */
int trans_ev_tridi_to_band_d(int64_t n, int nbw, int64_t nev,
                             const double *hh_v, const double *hh_tau,
                             double *Z, int64_t ldz,
                             void *work, size_t work_bytes, void *stream);

/* Complex FP64 (Hermitian problems); tau is complex as produced by the
 * standard complex Householder method.  Same contract as the real call. */
int trans_ev_tridi_to_band_z(int64_t n, int nbw, int64_t nev,
                             const trbt_z *hh_v, const trbt_z *hh_tau,
                             trbt_z *Z, int64_t ldz,
                             void *work, size_t work_bytes, void *stream);

/* The same operation in two steps, for callers that time or reuse them:
 *   trbt_prepare_*  precomputes, from hh_v/hh_tau only, the per-block
 *                   compact-WY factors into `work` (arguments as above:
 *                   1 n, 2 nbw, 3 hh_v, 4 hh_tau, 5 work, 6 work_bytes,
 *                   7 stream; work_bytes must be at least
 *                   trbt_workspace_bytes(n, nbw, n, is_complex));
 *   trbt_apply_*    applies them to Z (arguments exactly as for
 *                   trans_ev_tridi_to_band_*).
 * apply must follow a prepare of the same (n, nbw, hh_v, hh_tau contents)
 * on the same workspace, ordered on the stream; one prepare can serve any
 * number of applies to different Z (the factors depend on the reflectors
 * only).  trans_ev_tridi_to_band_* is exactly prepare followed by apply. */
int trbt_prepare_d(int64_t n, int nbw, const double *hh_v, const double *hh_tau,
                   void *work, size_t work_bytes, void *stream);
int trbt_prepare_z(int64_t n, int nbw, const trbt_z *hh_v, const trbt_z *hh_tau,
                   void *work, size_t work_bytes, void *stream);
int trbt_apply_d(int64_t n, int nbw, int64_t nev, const double *hh_v, const double *hh_tau,
                 double *Z, int64_t ldz, void *work, size_t work_bytes, void *stream);
int trbt_apply_z(int64_t n, int nbw, int64_t nev, const trbt_z *hh_v, const trbt_z *hh_tau,
                 trbt_z *Z, int64_t ldz, void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Adjoint (reverse-mode derivative) of the real back-transformation.
 * With Z_out = H_0 H_1 ... H_{K-1} Z_in (Eq. 2stage_bkwd1, real reflectors
 * H_k = I - tau_k v_k v_k^T) and G = dL/dZ_out for some scalar L, it returns
 *   dL/dZ_in = H_{K-1}^T ... H_0^T G        (in place in G),
 *   dL/dv    (K x nbw, row k = reflector k, zero beyond its length),
 *   dL/dtau  (K).
 * The intermediate states of the forward pass are recomputed from
 * checkpoints taken every 16 stages (of the band's bulge-chasing stages,
 * Sec. 2.2.1) by a first forward pass over a scratch copy of Z_in; the
 * column sums that form dL/dv and dL/dtau are reduced in a fixed order, so
 * results are bitwise reproducible.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for the adjoint of (n, nbw, nev); ckpt_every is 0 or 16
 * (the default, and the only interval implemented).  Errors: -1 n, -2 nbw,
 * -3 nev, -4 ckpt_every, -5 null `bytes`.  The workspace is large: the
 * checkpoints hold about n^2/(2 nbw) * (nbw + 16) * nev / 16 doubles, and
 * the backward pass saves the gradient windows in as many again. */
int trbt_adjoint_workspace_bytes_d(int64_t n, int nbw, int64_t nev, int ckpt_every,
                                   size_t *bytes);

/* Arguments: 1 n >= 0, 2 nbw in [1, TRBT_NBW_MAX], 3 0 <= nev <= n,
 * 4 hh_v, 5 hh_tau (device, as for the forward call), 6 Z_in (device,
 * n x nev column-major, read only), 7 ldz >= max(1, n), 8 G (device,
 * n x nev column-major: dL/dZ_out on entry, dL/dZ_in on exit),
 * 9 ldg >= max(1, n), 10 dv (device, K x nbw, written entirely), 11 dtau
 * (device, K), 12 ckpt_every (0 or 16), 13 work (device, aligned to
 * TRBT_WORK_ALIGN), 14 work_bytes (at least trbt_adjoint_workspace_bytes_d),
 * 15 stream.  Pointers may be NULL where nothing is read or written
 * (K == 0, or nev == 0 for Z_in and G).  K == 0 returns without touching
 * anything (dL/dZ_in = G); nev == 0 sets dv and dtau to zero.
 * Asynchronous on `stream`; no allocation.  Returns TRBT_ERR_WORKSPACE when
 * work is missing or too small. */
int trans_ev_tridi_to_band_adjoint_d(int64_t n, int nbw, int64_t nev,
                                     const double *hh_v, const double *hh_tau,
                                     const double *Z_in, int64_t ldz,
                                     double *G, int64_t ldg,
                                     double *dv, double *dtau, int ckpt_every,
                                     void *work, size_t work_bytes, void *stream);

/* The same adjoint in two halves, for callers (such as an autograd
 * framework) that run the forward transformation anyway and keep the
 * checkpoints until the backward pass instead of recomputing them:
 *   trans_ev_tridi_to_band_fwd_ckpt_d  Z <- Q^* Z in place (the same result,
 *       bitwise, as trans_ev_tridi_to_band_d) and writes the checkpoints
 *       into `work`.  Arguments: 1 n, 2 nbw, 3 nev, 4 hh_v, 5 hh_tau, 6 Z,
 *       7 ldz, 8 ckpt_every (0 or 16), 9 work, 10 work_bytes, 11 stream.
 *   trans_ev_tridi_to_band_bwd_ckpt_d  G <- dL/dZ_in and dv, dtau from the
 *       checkpoints a previous fwd_ckpt call with the same n, nbw, nev and
 *       reflectors left in `work` (ordered before it on the stream; work
 *       untouched in between).  Arguments: 1 n, 2 nbw, 3 nev, 4 hh_v,
 *       5 hh_tau, 6 G, 7 ldg, 8 dv, 9 dtau, 10 ckpt_every, 11 work,
 *       12 work_bytes, 13 stream.
 * Workspace size: trbt_adjoint_workspace_bytes_d.  Same validation rules and
 * status codes as the one-call adjoint. */
int trans_ev_tridi_to_band_fwd_ckpt_d(int64_t n, int nbw, int64_t nev,
                                      const double *hh_v, const double *hh_tau,
                                      double *Z, int64_t ldz, int ckpt_every,
                                      void *work, size_t work_bytes, void *stream);
int trans_ev_tridi_to_band_bwd_ckpt_d(int64_t n, int nbw, int64_t nev,
                                      const double *hh_v, const double *hh_tau,
                                      double *G, int64_t ldg, double *dv, double *dtau,
                                      int ckpt_every, void *work, size_t work_bytes,
                                      void *stream);

/* Adjoint of the complex back-transformation (H_k = I - tau_k v_k v_k^H,
 * complex tau) for a real scalar L, in the conjugate-Wirtinger convention:
 * every returned gradient grad_x satisfies dL = Re sum conj(grad_x) dx for
 * complex perturbations dx (the convention of PyTorch's complex autograd).
 * On entry G = grad of Z_out; on exit
 *   grad Z_in = H_{K-1}^H ... H_0^H G        (in place in G),
 *   grad v_k  = sum over columns of -conj(tau_k) conj(w) g - tau_k conj(gamma) z,
 *   grad tau_k = sum over columns of -conj(w) gamma,
 * with z the column rows entering H_k in the forward pass, g the gradient
 * rows leaving it, w = v_k^H z and gamma = v_k^H g.  For nbw in {16, 32,
 * 48, 64} the blocked form of the real adjoint with complex operands
 * (compact-WY blocks of 16 stages on FP64 MFMA, a checkpoint of every
 * block's input window, a gradient sweep and a per-block reduction);
 * workspace: a copy of Z_in, the packed factors of both passes and two
 * copies of every block's (nbw+16) x 16 windows, about
 * n^2 nev (nbw+16) / nbw bytes in all (43 GB at n = 4096, nbw = 64,
 * nev = 2048).  Other nbw: stage by
 * stage (the slots of a stage are disjoint, Sec. 2.2.2: one launch per
 * stage over all slots and columns) on row-major working copies of Z and G,
 * with the rows a 16-stage segment touches checkpointed before it and the
 * segment recomputed in the reverse sweep; workspace: two working copies,
 * the checkpoints (about n^2 nev / 32 complex), one segment's tape and
 * per-256-column partial sums.  Both forms take the column sums behind dv
 * and dtau in a fixed order (bitwise reproducible).
 * Arguments, validation and status codes as trans_ev_tridi_to_band_adjoint_d,
 * with complex hh_v, hh_tau, Z_in, G, dv, dtau and the workspace size from
 * trbt_adjoint_workspace_bytes_z. */
int trbt_adjoint_workspace_bytes_z(int64_t n, int nbw, int64_t nev, int ckpt_every,
                                   size_t *bytes);
int trans_ev_tridi_to_band_adjoint_z(int64_t n, int nbw, int64_t nev,
                                     const trbt_z *hh_v, const trbt_z *hh_tau,
                                     const trbt_z *Z_in, int64_t ldz,
                                     trbt_z *G, int64_t ldg,
                                     trbt_z *dv, trbt_z *dtau, int ckpt_every,
                                     void *work, size_t work_bytes, void *stream);

/* The complex adjoint in two halves, like the real pair above (the same
 * reverse-mode definition, conjugate-Wirtinger gradients), for nbw in
 * {16, 32, 48, 64}:
 *   trans_ev_tridi_to_band_fwd_ckpt_z  Z <- Q^* Z in place (bitwise the
 *       result of trans_ev_tridi_to_band_z) and the checkpoints into `work`.
 *       Arguments: 1 n, 2 nbw, 3 nev, 4 hh_v, 5 hh_tau, 6 Z, 7 ldz,
 *       8 ckpt_every (0 or 16), 9 work, 10 work_bytes, 11 stream.
 *   trans_ev_tridi_to_band_bwd_ckpt_z  G <- grad Z_in and dv, dtau (bitwise
 *       those of trans_ev_tridi_to_band_adjoint_z) from the checkpoints a
 *       previous fwd_ckpt_z call with the same n, nbw, nev and reflectors
 *       left in `work` (ordered before it on the stream; work untouched in
 *       between).  Arguments: 1 n, 2 nbw, 3 nev, 4 hh_v, 5 hh_tau, 6 G,
 *       7 ldg, 8 dv, 9 dtau, 10 ckpt_every, 11 work, 12 work_bytes, 13 stream.
 * Complex hh_v, hh_tau, Z, G, dv, dtau; ldz, ldg in complex elements;
 * workspace size: trbt_adjoint_workspace_bytes_z.  Status codes as the real
 * pair, and -2 for any other nbw (those band widths have only the one-call
 * complex adjoint), -1 also for n beyond the blocked kernels' range. */
int trans_ev_tridi_to_band_fwd_ckpt_z(int64_t n, int nbw, int64_t nev,
                                      const trbt_z *hh_v, const trbt_z *hh_tau,
                                      trbt_z *Z, int64_t ldz, int ckpt_every,
                                      void *work, size_t work_bytes, void *stream);
int trans_ev_tridi_to_band_bwd_ckpt_z(int64_t n, int nbw, int64_t nev,
                                      const trbt_z *hh_v, const trbt_z *hh_tau,
                                      trbt_z *G, int64_t ldg, trbt_z *dv, trbt_z *dtau,
                                      int ckpt_every, void *work, size_t work_bytes,
                                      void *stream);

/* ------------------------------------------------------------------------
 * Batched back-transformation: many independent problems of uneven size
 * (k-points, spin channels), all real or all complex, each exactly the
 * operation above, run through one persistent launch per band width,
 * captured once in a HIP graph.
 * ------------------------------------------------------------------------ */

/* One problem: the arguments of trans_ev_tridi_to_band_d.  All pointers are
 * device pointers owned by the caller.  Distinct problems must not share
 * Z storage. */
typedef struct {
    int64_t n;
    int nbw;
    int64_t nev;
    const double *hh_v;
    const double *hh_tau;
    double *Z;
    int64_t ldz;
} trbt_problem_d;

/* Launch configuration of a plan.
 *   strip_cols    columns of Z per workgroup task: 16 or 32;
 *   waves         wavefronts per workgroup (slots in flight): 4 or 8;
 *   block_stages  16: compact-WY blocks of 16 consecutive stages on FP64
 *                 MFMA (problems with nbw in {16, 32, 48, 64}; other nbw
 *                 fall back to the streaming form); 1: every problem with
 *                 the streaming form, one reflector at a time, one lane per
 *                 column (strip_cols and waves then do not matter). */
typedef struct {
    int strip_cols;
    int waves;
    int block_stages;
} trbt_plan_config;

/* One complex problem: the arguments of trans_ev_tridi_to_band_z.  A plan
 * holds real problems only (trbt_plan_create_batched_d) or complex problems
 * only (trbt_plan_create_batched_z). */
typedef struct {
    int64_t n;
    int nbw;
    int64_t nev;
    const trbt_z *hh_v;
    const trbt_z *hh_tau;
    trbt_z *Z;
    int64_t ldz;
} trbt_problem_z;

typedef struct trbt_plan trbt_plan;   /* opaque */

/* Status of a problem descriptor that fails the single-call checks. */
#define TRBT_ERR_PROBLEM(i) (-1000 - (i))

/* Create a plan for `count` problems on the current device.
 * Arguments: 1 probs (host array, copied; non-NULL unless count == 0),
 * 2 count >= 0, 3 cfg (host; NULL = autotune, see below; otherwise checked
 * against the values listed above), 4 plan (out, set to NULL on failure),
 * 5 stream.  Descriptor i failing the checks of trans_ev_tridi_to_band_d
 * returns TRBT_ERR_PROBLEM(i).
 * Blocking call: it synchronizes `stream` (which may still be producing the
 * inputs), allocates the plan's device memory (header, packed compact-WY
 * blocks of every problem, task tables; the only allocation of the plan's
 * life) and captures the launch sequence into a graph.  With cfg == NULL it
 * first times every candidate configuration on device scratch copies of the
 * problems' Z (freed before returning) and keeps the fastest; the caller's
 * Z is not modified.  Candidates: strip_cols 16/32 x waves 4/8 with
 * block_stages 16, and block_stages 1 when no problem can take the blocked
 * form or every problem has n <= 256.
 * Tuning cache: when the environment variable TRBT_TUNE_CACHE names a file,
 * a tuned plan's choice is appended to it as one text line keyed by the
 * problem set's signature (device architecture and CU count, real or
 * complex, the sorted (n, nbw, nev) of all problems -- not the pointers),
 * and a later cfg == NULL plan with the same signature takes it from there
 * without timing (trbt_plan_get_config then reports the cached time).  An
 * unreadable or unwritable file only means tuning runs as without it. */
int trbt_plan_create_batched_d(const trbt_problem_d *probs, int count,
                               const trbt_plan_config *cfg, trbt_plan **plan,
                               void *stream);

/* The same for complex Hermitian problems (the operation of
 * trans_ev_tridi_to_band_z per problem).  Complex plans use 16-column
 * strips: strip_cols 32 is rejected (-3) and not among the tuning
 * candidates.  Arguments and status codes otherwise as above. */
int trbt_plan_create_batched_z(const trbt_problem_z *probs, int count,
                               const trbt_plan_config *cfg, trbt_plan **plan,
                               void *stream);

/* Run the plan on `stream`: every problem's Z <- Q_i^* Z, in place.
 * The plan keeps the descriptors and pointers given at creation: buffer
 * contents (Z, hh_v, hh_tau) may change between executions, addresses may
 * not.  Executions of one plan must not overlap in time (they share the
 * plan's device state); ordering them on one stream is enough.
 * Errors: -1 null plan, TRBT_ERR_DEVICE (another device is current),
 * TRBT_ERR_HIP. */
int trbt_plan_exec(trbt_plan *plan, void *stream);

/* The configuration in use and, if tuned, the best measured time of one
 * execution in milliseconds (0 when the configuration was given). */
int trbt_plan_get_config(const trbt_plan *plan, trbt_plan_config *cfg, double *tuned_ms);

/* Synchronize the device and report the plan's fault word: 0 when every
 * bounded inter-wave wait of the last execution completed (nonzero never
 * expected; the results are then invalid). */
int trbt_plan_check(trbt_plan *plan, int *fault);

/* Free the plan (synchronizes the device first).  NULL is accepted. */
int trbt_plan_destroy(trbt_plan *plan);

/* ------------------------------------------------------------------------
 * Banded-to-tridiagonal reduction (the producer of hh_v / hh_tau)
 *
 * Bulge chasing, Sec. 2.2.1, Eq. 2stage_fwd2, with reflectors built as in
 * Eq. householder: for stage s = 0 .. n-3 and sweep j = 0 .. S_s-1, the
 * reflector H = I - tau v v^H with v[0] = 1 and H^H x = beta e1 (beta real,
 * beta = -sign(Re x0) ||x||, tau = 0 and v = e1 when x has nothing to
 * annihilate) is built from column c of the current matrix on rows
 * [r0, r0+len) (c = s for j = 0, else c = r0 - nbw: the first column of the
 * bulge left by sweep j-1), and B <- H^H B H.  The reflectors come out in
 * generation order, exactly the layout trans_ev_tridi_to_band_{d,z} take,
 * so that  B = Q T Q^H  with Q^* = H_0 H_1 ... H_{K-1} as above.
 *
 * Stages run as a pipeline on the GPU: stage s takes sweep j once stage s-1
 * has finished sweep j+2; the result equals the sequential order's up to
 * rounding (the same operations on the same data; only the summation order
 * inside a step differs).
 * ------------------------------------------------------------------------ */

/* Bytes of device workspace trbt_band_to_tridi_{d,z} need: the band with
 * 2*nbw stored diagonals (the chase's fill) and one progress counter per
 * stage.  Errors: -1 n < 0, -2 nbw outside [1, 64], -4 null `bytes`. */
int trbt_band_to_tridi_workspace_bytes(int64_t n, int nbw, int is_complex, size_t *bytes);

/* Reduce the Hermitian band matrix B (n x n, semi-bandwidth nbw) to the
 * real symmetric tridiagonal T = diag(d) + subdiag(e) (complex case: e is
 * complex; after the last stage only e[n-2] keeps a nonzero imaginary part),
 * writing the reflectors.
 * Arguments: 1 n in [0, 2^30] (the chase's progress counters are 32-bit;
 * -1 outside), 2 nbw in [1, 64], 3 ab (device, read-only): B in
 * LAPACK lower band layout, ab[d + k*ldab] = B(k+d, k) for d = 0..nbw
 * (entries with k+d >= n ignored; imaginary parts of the diagonal ignored
 * in the complex case), 4 ldab >= nbw+1, 5 d (device, n reals, out),
 * 6 e (device, n-1 entries, out), 7 hh_v (device, K x nbw, out; entries at
 * positions >= len_k written as zero), 8 hh_tau (device, K, out), 9 work
 * (device, aligned to TRBT_WORK_ALIGN), 10 work_bytes (at least
 * trbt_band_to_tridi_workspace_bytes), 11 stream.  K =
 * trbt_num_reflectors(n, nbw); hh_v / hh_tau may be NULL when K == 0 (n < 3
 * or nbw == 1: the band is already tridiagonal and only d, e are written).
 * Asynchronous on `stream`, no allocation; TRBT_ERR_WORKSPACE when work is
 * missing or too small.  Successive calls on one workspace must be ordered
 * (one stream is enough).  If a pipeline wait ever timed out (never
 * expected; a 10 s bound per wait), d is filled with NaN. */
int trbt_band_to_tridi_d(int64_t n, int nbw, const double *ab, int64_t ldab, double *d,
                         double *e, double *hh_v, double *hh_tau, void *work,
                         size_t work_bytes, void *stream);
int trbt_band_to_tridi_z(int64_t n, int nbw, const trbt_z *ab, int64_t ldab, double *d,
                         trbt_z *e, trbt_z *hh_v, trbt_z *hh_tau, void *work,
                         size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Tridiagonal eigenpairs (the step between the chase and the
 * back-transformation, Eq. 2stage_solve): the lowest nev eigenvalues of the
 * real symmetric tridiagonal T = diag(d) + subdiag(e), ascending, and their
 * eigenvectors, computed only for the wanted ones -- eigenvalue i by
 * bisection on the Sturm count, eigenvector i by inverse iteration (pivoted
 * tridiagonal LU, a fixed pseudo-random start, two solves), one GPU thread
 * per eigenpair.  Each eigenvector is normalised with its largest-magnitude
 * entry positive (except vectors of a cluster after its orthonormalisation).
 * Accuracy: residuals ||T z - w z|| ~ eps ||T||; the angle between the
 * vectors of eigenvalues a gap apart ~ eps ||T|| / gap; eigenvalues within
 * 1e-6 ||T|| of each other form a cluster whose vectors are orthonormalised
 * together (modified Gram-Schmidt), so degenerate eigenvalues get an
 * orthonormal basis of their eigenspace.
 * For the complex chase's T (every subdiagonal a real beta except e[n-2])
 * pass Re e with its last entry replaced by |e[n-2]| and multiply the last
 * row of Z by e[n-2] / |e[n-2]| afterwards (T = D T_r D^H with
 * D = diag(1, ..., 1, e[n-2] / |e[n-2]|)).
 * ------------------------------------------------------------------------ */

/* Workspace bytes: about n * nev * 41 (the iterates, the LU factors and the
 * pivot flags).  Errors: -1 n < 0, -2 nev outside [0, n], -3 null `bytes`. */
int trbt_tridiag_eigh_workspace_bytes(int64_t n, int64_t nev, size_t *bytes);

/* Arguments: 1 n >= 0, 2 0 <= nev <= n, 3 d (device, n), 4 e (device, n-1),
 * 5 w (device, nev, out: eigenvalues ascending), 6 Z (device, n x nev
 * column-major, out), 7 ldz >= max(1, n), 8 work (device, aligned to
 * TRBT_WORK_ALIGN), 9 work_bytes (at least trbt_tridiag_eigh_workspace_bytes),
 * 10 stream.  nev == 0 returns at once.  Asynchronous on `stream`; no
 * allocation; TRBT_ERR_WORKSPACE when work is missing or too small. */
int trbt_tridiag_eigh_d(int64_t n, int64_t nev, const double *d, const double *e, double *w,
                        double *Z, int64_t ldz, void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Band-to-full back-transformation (the step after the tridiagonal-to-
 * banded one; Sec. 2.1, Eq. 2stage_bkwd2):
 *
 *     C = P^* Y,   P^* = H_0 H_1 ... H_{J-1},   H_j = I - tau_j v_j v_j^H,
 *
 * where B = P A P^* (Eq. 2stage_fwd1) is the full-to-band reduction of the
 * Hermitian A with one reflector per column: v_j acts on rows [j+nbw, n)
 * (j = 0 .. J-1, J = max(0, n-nbw-1)) and annihilates column j below the
 * band.  The reflectors are applied in reverse generation order, each as
 * y <- y - tau_j v_j (v_j^H y) on its rows (the operation of Eq. kernel);
 * the library merges 64 consecutive reflectors into one compact-WY factor
 * I - V T V^H and applies it with dense products on FP64 MFMA.
 *
 * Data layout:
 *   hh_v    n x J, column-major, leading dimension ldv >= max(1, n):
 *           column j holds v_j in rows [j+nbw, n), v_j[0] at row j+nbw
 *           (read, not assumed to be 1).  Rows above j+nbw of column j and
 *           rows n .. ldv-1 are never read (LAPACK keeps such reflectors
 *           below the band of the reduced matrix; any storage with this
 *           shape works).
 *   hh_tau  J scalars.
 *   Z       n x nev column-major (ldz >= max(1, n)), overwritten with C;
 *           rows n .. ldz-1 are never read or written.
 * ------------------------------------------------------------------------ */

/* Workspace bytes: 256 + ceil(J/64) * 64 * 64 scalars (the per-panel
 * compact-WY factors T); 0 when J == 0 or nev == 0.  Errors: -1 n < 0,
 * -2 nbw < 1, -3 nev outside [0, n], -4 null `bytes`. */
int trbt_band_to_full_workspace_bytes(int64_t n, int nbw, int64_t nev, int is_complex,
                                      size_t *bytes);

/* Arguments: 1 n >= 0, 2 nbw >= 1, 3 0 <= nev <= n, 4 hh_v (device, non-null
 * unless J == 0 or nev == 0), 5 ldv >= max(1, n), 6 hh_tau (device, J),
 * 7 Z (device, non-null unless nev == 0 or n == 0), 8 ldz >= max(1, n),
 * 9 work (device, aligned to TRBT_WORK_ALIGN), 10 work_bytes (at least
 * trbt_band_to_full_workspace_bytes), 11 stream.  J == 0 (n <= nbw+1) or
 * nev == 0 return TRBT_SUCCESS without touching Z.  Asynchronous on
 * `stream`, no allocation; TRBT_ERR_WORKSPACE when work is missing or too
 * small.  The kernels have no waits between workgroups (the fault word
 * stays clear).  Results are bitwise reproducible. */
int trans_ev_band_to_full_d(int64_t n, int nbw, int64_t nev, const double *hh_v, int64_t ldv,
                            const double *hh_tau, double *Z, int64_t ldz, void *work,
                            size_t work_bytes, void *stream);
int trans_ev_band_to_full_z(int64_t n, int nbw, int64_t nev, const trbt_z *hh_v, int64_t ldv,
                            const trbt_z *hh_tau, trbt_z *Z, int64_t ldz, void *work,
                            size_t work_bytes, void *stream);

/* Allocation-free form of trans_ev_band_to_full_z, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same operation,
 * arguments 1-8 and results (bitwise) as trans_ev_band_to_full_z; argument
 * 9 is the stream.  The compact-WY factors go to a fixed device array of
 * TRBT_B2F_SCRATCH_BYTES inside the library (one per device the library
 * runs on, held until the process ends), so the call allocates nothing.
 * It takes problems whose workspace (trbt_band_to_full_workspace_bytes,
 * is_complex = 1) fits in that array -- with 64-reflector panels, J =
 * n - nbw - 1 <= 32704 -- and returns TRBT_ERR_SCRATCH for larger ones
 * before any launch.  All calls on one device share the array: calls that
 * may overlap in time on one device (different streams, or several host
 * threads without ordering) race on it and give wrong results; calls
 * ordered on one stream are safe.  The first call on each device looks up
 * the array's device address (hipGetSymbolAddress) with that device current. */
#define TRBT_B2F_SCRATCH_BYTES (32u << 20)
int trans_ev_band_to_full_z_noalloc(int64_t n, int nbw, int64_t nev, const trbt_z *hh_v,
                                    int64_t ldv, const trbt_z *hh_tau, trbt_z *Z, int64_t ldz,
                                    void *stream);

/* Fault word of a workspace.  The blocked kernels of
 * trans_ev_tridi_to_band_{d,z} / trbt_apply_{d,z}, of the real adjoints
 * (trans_ev_tridi_to_band_adjoint_d, _fwd_ckpt_d, _bwd_ckpt_d) and of the
 * complex adjoint keep 32 bits at offset 0 of their workspace: clear after
 * trbt_prepare_*, at the start of a one-call transform or adjoint and at
 * the start of fwd_ckpt (bwd_ckpt keeps it, so a pair reports both halves),
 * set when a bounded wait between workgroups gave up (never expected; the
 * outputs of that call -- Z, or G, dv, dtau -- are then INVALID although
 * the call returned TRBT_SUCCESS).
 * Arguments: 1 work (device, the workspace of such a call, aligned to
 * TRBT_WORK_ALIGN; NULL when the call ran without one -- the streaming
 * kernels have no waits -- which gives *fault = 0), 2 fault (host, out:
 * 0 or 1), 3 stream (the stream the call ran on).
 * Blocking: it synchronizes `stream` and then reads the word.  The word of
 * the banded-to-tridiagonal workspace is not this one (that call reports a
 * timeout by filling d with NaN).  Errors: -1 misaligned work, -2 null
 * fault, TRBT_ERR_HIP. */
int trbt_work_check(const void *work, int *fault, void *stream);

/* Static description of a status code (never NULL). */
const char *trbt_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* TRBT_H */
