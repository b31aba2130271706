/*
 * mlfma.h -- C ABI of the MI355X (gfx950) MLFMA matvec for the Helmholtz
 * potential
 *
 *     phi_i = sum_{j != i} q_j exp(i k |r_i - r_j|) / |r_i - r_j|,
 *
 * the pair-potential sum of the paper's problem statement (Sec. 2, Eq. for
 * Phi(r)) with the kernel written exp(+ikr)/r (the paper's exp(-jkr)/(4 pi r)
 * is its complex conjugate over 4 pi for real k; the adjoint entry point
 * evaluates that convention up to the 1/(4 pi) factor).
 *
 * The library evaluates it with the multilevel fast multipole algorithm of
 * the paper: an octree over the points (Sec. 2 FMM paragraph, Sec. 3.1),
 * leaf plane-wave signatures (C2M, Sec. 3.2.1), interpolation + shift +
 * aggregation up the tree (M2M, Sec. 3.2.2), diagonal translation over the
 * far-field lists (M2L, Sec. 3.2.3), shift + anterpolation + aggregation down
 * the tree (L2L, Sec. 3.2.4), evaluation at the leaf points (L2O, Sec. 3.2.5)
 * and the direct near-field sum at the leaf level (Sec. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status: MLFMA_OK (0) on success, a positive MLFMA_E* code otherwise.
 *   The library never aborts and never prints; mlfma_last_error() returns a
 *   thread-local text for the last failing call on the calling thread.
 * - Host pointers are read during the call only; the library keeps copies.
 * - Device pointers are caller-owned HIP device buffers on the device the
 *   tree was built for.  Work is enqueued on `stream` (a hipStream_t, NULL =
 *   the null stream) and is NOT complete when the call returns; the caller
 *   synchronises the stream before reading results.
 * - Complex arrays are interleaved (re, im); dtype MLFMA_C64 = float pairs,
 *   MLFMA_C128 = double pairs (converted to and from FP32 inside the
 *   kernels; the arithmetic is FP32 either way).
 * - Per-point arrays are in the CALLER's point order, row-major
 *   [n][nrhs] (column c = right-hand side c).
 * - An operator handle owns one workspace: calls on one handle must not
 *   overlap in time (different handles may run concurrently).
 */
#ifndef MLFMA_H
#define MLFMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlfma_tree_s *mlfma_tree_t;
typedef struct mlfma_ops_s *mlfma_ops_t;

enum mlfma_status {
    MLFMA_OK = 0,
    MLFMA_EINVAL = 1,  /* invalid argument (null pointer, bad size, NaN, ...) */
    MLFMA_EDEPTH = 2,  /* tree deeper than max_levels or than 21 levels      */
    MLFMA_ENOMEM = 3,  /* host or device allocation failed / over the limit  */
    MLFMA_EDEVICE = 4, /* HIP runtime error (no device, launch failure, ...) */
    MLFMA_ERANGE = 5   /* moved point left its box (mlfma_update_positions) */
};

enum mlfma_dtype { MLFMA_C64 = 0, MLFMA_C128 = 1 };

/* parts of the matvec to evaluate (mlfma_matvec_ex) */
enum mlfma_parts {
    MLFMA_NEAR = 1, /* direct sum over near-field leaves                    */
    MLFMA_FAR = 2,  /* C2M, M2M, M2L, L2L, L2O                               */
    MLFMA_CONJ = 4  /* conjugate input and output: A^H v (adjoint)           */
};

/* mlfma_precompute_operators flags */
enum mlfma_flags {
    MLFMA_FP32 = 0,          /* FP32 interpolation / anterpolation GEMMs     */
    MLFMA_BF16X3_INTERP = 1, /* interpolation GEMMs in BF16 split precision
                                (hi*hi + hi*lo + lo*hi, FP32 accumulation)  */
    MLFMA_NO_AUTOTUNE = 2,   /* skip the kernel-variant timing at precompute
                                (variants differ only in summation order;
                                the timing takes each form alone, then
                                searches the concurrent schedule with the
                                close forms inside the whole step, about
                                5 s for 262k points at one RHS)             */
    MLFMA_USE_GRAPH = 4,     /* capture each distinct call (buffers, nrhs,
                                dtype, parts, stream) into a HIP graph once
                                and replay it afterwards; calls on the null
                                stream and profiled calls run eagerly       */
    MLFMA_ONE_STREAM = 8,    /* run every kernel on the caller's stream (by
                                default the near field and the M2L of each
                                level run on two library streams, forked
                                from and joined back to the caller's stream
                                with events, so they overlap the M2M chain) */
    MLFMA_SAMPLED_OPERATORS = 16 /* keep the translation operators as sampled
                                tables instead of their values at every grid
                                direction (Sec. 3.2.3 "Translation Operators":
                                sample and interpolate when memory is short):
                                per distinct offset length, T at 8 L + 1
                                angles to the offset; M2L interpolates its
                                operators (10-point Lagrange, relative error
                                below 3e-8) into LDS; M2L forms 3, 4, 5 and 9
                                only */
};

typedef struct mlfma_tree_info {
    int64_t n_points;
    int32_t n_levels;    /* root = level 1, leaves = level n_levels          */
    int32_t device;
    double leaf_size;    /* side of a leaf box                               */
    double root_size;    /* D0 = leaf_size * 2^(n_levels-1)                  */
    double origin[3];    /* lowest corner of the root cube                   */
    int64_t n_leaf_boxes;
    int64_t n_near_pairs; /* sum over leaves of |near list| (incl. self)      */
    int64_t n_p2p_pairs;  /* point pairs of the near field (incl. i = j)      */
} mlfma_tree_info;

typedef struct mlfma_level_info {
    int32_t level;
    int32_t L;          /* truncation order (0 if the level has no spectra)  */
    int32_t ntheta;     /* L + 1 Gauss-Legendre nodes in cos(theta)          */
    int32_t nphi;       /* 2L + 2 uniform samples in phi                     */
    int64_t K;          /* ntheta * nphi samples per box                     */
    int64_t nbox;       /* non-empty boxes at this level                     */
    int64_t n_far;      /* far-field (observer, source) pairs at this level  */
    int32_t n_types;    /* distinct translation offsets used                 */
    int32_t pad;
} mlfma_level_info;

/*
 * Build the octree (host only; no device call is made here).
 * Sec. 3.1: n_levels is the smallest integer with
 * leaf_size * 2^(n_levels-1) >= E, E the largest side of the points'
 * bounding box; the root cube (side D0 = leaf_size * 2^(n_levels-1)) is
 * centred on the bounding box.  A point's leaf box is
 * floor((r - origin) / leaf_size) per axis, clamped into the cube; its box at
 * level l is that index shifted right by n_levels - l; empty boxes are
 * dropped; boxes and points are kept in Morton-Z order (ties by input index).
 * Near field (leaf level): Chebyshev distance <= 1 (Sec. 2).  Far field at
 * level l >= 3: not near, parents near (Sec. 2).
 *
 *   xyz        host, [n][3] doubles, caller order
 *   n          >= 0 (n = 0 gives an empty tree; every matvec is a no-op)
 *   leaf_size  > 0, finite
 *   max_levels 1..21
 *   device     HIP device ordinal used by mlfma_precompute_operators
 *   out        receives the handle (owned by the caller; mlfma_destroy_tree)
 * Errors: EINVAL (null pointer, n < 0, non-finite coordinate, bad leaf_size
 *         or max_levels), EDEPTH, ENOMEM.
 */
int mlfma_build_tree(const double *xyz, int64_t n, double leaf_size,
                     int max_levels, int device, mlfma_tree_t *out);

/*
 * Replace the point coordinates while keeping the tree's topology (used for
 * finite-difference checks of position gradients).  Every point must stay
 * inside the root cube and in its leaf box (same floor index); otherwise
 * ERANGE and nothing changes.  Existing handles wait for the device to be
 * idle before their next call uploads the new positions.
 * Takes effect for operator handles created afterwards and, for existing
 * handles, at their next call (the device copy is refreshed lazily).
 */
int mlfma_update_positions(mlfma_tree_t t, const double *xyz);

/*
 * Precompute everything a matvec needs, in FP64 on the host, and upload it
 * (FP32 / complex64 tables) with the tree to the tree's device.  Per level
 * l >= 3 the truncation order is
 *     L = ceil(k d + 1.8 digits^(2/3) (k d)^(1/3)),  d = sqrt(3) a_l,
 * samples are Gauss-Legendre in cos(theta) x 2L+2 uniform in phi, the
 * translation operator of offset X is
 *     T(khat) = sum_{l<=L} i^l (2l+1) h_l^(1)(k|X|) P_l(khat . X/|X|)
 * (Sec. 3.2.3, translation operators, precomputed once), and the level-to-
 * level maps are the exact band-limited interpolation (Sec. 2 related work,
 * global interpolation; Sec. 3.2.2) and its weighted adjoint.
 * Also allocates the workspace for up to max_rhs right-hand sides; matvec
 * calls allocate nothing.
 *
 *   k       wavenumber > 0
 *   digits  1..10 (3 = about three digits)
 *   max_rhs 1..1024
 *   flags   MLFMA_FP32 or MLFMA_BF16X3_INTERP
 * Errors: EINVAL (k <= 0 or non-finite, digits, max_rhs, flags, a leaf box
 *         with k sqrt(3) leaf_size < 1 while the tree has far-field levels --
 *         the diagonal form is not accurate there -- or a leaf box larger
 *         than about 72 wavelengths, k 2 sqrt(3) leaf_size / (2 pi) > 250,
 *         beyond the range of the near field's FP32 phase evaluation),
 *         ENOMEM (device memory or
 *         the limit of mlfma_set_device_memory_limit), EDEVICE.
 * The ops handle keeps a reference to the tree (destroying the tree first is
 * allowed).
 */
int mlfma_precompute_operators(mlfma_tree_t t, double k, int digits,
                               int max_rhs, uint32_t flags, mlfma_ops_t *out);

/*
 * phi = A q (near + far), A_ij = exp(ik|r_i-r_j|)/|r_i-r_j|, A_ii = 0.
 *   q, phi  device, [n][nrhs] complex in the caller's point order
 *   nrhs    1..max_rhs
 *   dtype   MLFMA_C64 or MLFMA_C128
 *   stream  hipStream_t or NULL
 * Errors: EINVAL (null handle/pointer with n > 0, nrhs, dtype), EDEVICE.
 */
int mlfma_matvec(mlfma_ops_t ops, const void *q, void *phi, int64_t nrhs,
                 int dtype, void *stream);

/*
 * psi = A^H v = conj(A conj(v)) -- the conjugate-wavenumber MLFMA.  The
 * discrete operator is symmetric (antipodal sample grids, anterpolation the
 * weighted adjoint of interpolation), so this is its exact adjoint up to
 * rounding.  Same arguments and errors as mlfma_matvec.
 */
int mlfma_matvec_adjoint(mlfma_ops_t ops, const void *v, void *psi,
                         int64_t nrhs, int dtype, void *stream);

/*
 * As mlfma_matvec, evaluating only the parts in `parts` (MLFMA_NEAR,
 * MLFMA_FAR, optionally MLFMA_CONJ).  parts must contain NEAR or FAR.
 */
int mlfma_matvec_ex(mlfma_ops_t ops, const void *q, void *phi, int64_t nrhs,
                    int dtype, uint32_t parts, void *stream);

/*
 * Gradient of the potential at every point with respect to that point's
 * position, self term excluded:
 *     grad[i][c][a] = sum_{j != i} q_j[c] d/dr_i,a G(r_i - r_j),
 *     grad G(r) = G(r) (ik - 1/|r|) r/|r|.
 * Near part direct; far part = L2O with the extra factor ik khat.
 *   q     device [n][nrhs] complex;  grad  device [n][nrhs][3] complex
 * With parts = MLFMA_CONJ (others ignored) evaluates conj of the field of
 * conj(q).  Same errors as mlfma_matvec.
 */
int mlfma_field(mlfma_ops_t ops, const void *q, void *grad, int64_t nrhs,
                int dtype, uint32_t parts, void *stream);

/*
 * Position gradient of a real loss through phi = A q (the chain rule of the
 * pair sum, with the tree topology fixed):
 *     out[i][a] = sum_c Re[ conj(g[i][c]) F_q(r_i)[c][a] + q[i][c] F_conj(g)(r_i)[c][a] ],
 * where F_x is the field of charges x (mlfma_field) and g = 2 dL/d conj(phi)
 * is the incoming gradient of phi (PyTorch's convention for complex
 * tensors).  For L = ||phi - t||^2, g = 2 (phi - t) and
 * out = 2 Re[conj(e) F_q + q F_conj(e)], e = phi - t.
 *   q, g  device [n][nrhs] complex (dtype);  out device [n][3] real
 *         (float for MLFMA_C64, double for MLFMA_C128), caller order
 * Uses two field evaluations and the handle's workspace.  Errors as
 * mlfma_matvec.
 */
int mlfma_position_gradient(mlfma_ops_t ops, const void *q, const void *g, void *out,
                            int64_t nrhs, int dtype, void *stream);

/* NULL is a no-op.  Wait for outstanding work on the handle's streams first. */
/*
 * Iterative solve of the second-kind system (shift I + A) x = b, A the
 * potential operator of `ops` (phi = A q as mlfma_matvec computes it), for
 * one right-hand side: the iterative solver of the integral equations that
 * the potential sum comes from (Sec. 1, Sec. 2).  Restarted GMRES(restart)
 * (Saad and Schultz): Krylov basis in complex64 on the device, classical
 * Gram-Schmidt with FP64 coefficients (repeated when it cancels most of the
 * new vector), Givens rotations and the small least-squares problem on the
 * host in FP64.
 *   b, x       device, [n] complex64, caller order; x holds the initial
 *              guess on entry (zeros allowed) and the solution on exit.
 *              b and x must not overlap.
 *   shift      complex shift (shift_re + i shift_im) of the identity.
 *   restart    Krylov dimension per cycle, 1..500.
 *   max_iters  total operator applications allowed (0: only the residual
 *              of the initial guess is computed).
 *   tol        target ||b - (shift I + A) x|| / ||b|| (> 0).
 *   iters, rel_residual  host outputs (may be NULL): operator applications
 *              used, and the relative residual of the returned x,
 *              recomputed with the operator (not the GMRES estimate).
 * Not converging within max_iters is not an error: MLFMA_OK is returned and
 * rel_residual tells.  Synchronises `stream` (the residual checks run on the
 * host).  The workspace ((restart + 2) n complex64 and small buffers) is
 * allocated on the first call that needs it and kept by the handle; it is
 * counted against mlfma_set_device_memory_limit.
 * Errors: MLFMA_EINVAL (null or aliased buffers, restart, tol, shift),
 * MLFMA_ENOMEM, MLFMA_EDEVICE.
 */
int mlfma_solve_gmres(mlfma_ops_t ops, const void *b, void *x, double shift_re,
                      double shift_im, int restart, int max_iters, double tol,
                      int *iters, double *rel_residual, void *stream);

/* Bytes of device scratch behind mlfma_solve_gmres_noalloc, per GPU. */
#define MLFMA_GMRES_SCRATCH_BYTES (64ll << 20)

/*
 * mlfma_solve_gmres for callers that cannot allocate device memory (code
 * under HIP graph capture elsewhere in the process, serving loops or
 * harnesses that forbid hipMalloc): the same solve, arguments, results and
 * errors, but the Krylov basis, work vector, partial sums and coefficients
 * live in a fixed device array of MLFMA_GMRES_SCRATCH_BYTES (64 MiB) that
 * the library's code object holds on every GPU it runs on until the
 * process ends.  Nothing is allocated or freed on the device (the handle's
 * own matvec workspace, allocated by mlfma_precompute_operators, is used
 * as by every matvec).
 * Size limit: (restart + 2) n complex64 plus (restart + 1) (nb + 1)
 * complex FP64, nb = min(512, ceil(n / 2048)), each of the four buffers
 * rounded up to 256 bytes, must fit in MLFMA_GMRES_SCRATCH_BYTES (for
 * n = 262,144: restart up to 29); larger requests return MLFMA_ENOMEM
 * before any work is enqueued.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on the same GPU (other threads, other handles, other streams) race and
 * must be serialised by the caller.  The array keeps the last call's
 * contents; the solve initialises everything it reads.
 */
int mlfma_solve_gmres_noalloc(mlfma_ops_t ops, const void *b, void *x, double shift_re,
                              double shift_im, int restart, int max_iters, double tol,
                              int *iters, double *rel_residual, void *stream);

void mlfma_destroy_ops(mlfma_ops_t ops);
void mlfma_destroy_tree(mlfma_tree_t t);

/*
 * FFT interpolation / anterpolation between uniform sphere grids: the
 * paper's M2M interpolation (Sec. 3.2.2, paragraph "Fine-grained Parallel
 * Interpolation", Fig. 3: FFT interpolation along phi, then theta folded
 * into whole circles and FFT-interpolated along them) and the reverse used
 * in L2L (Sec. 3.2.4), as a batched operator, independent of any tree.
 *
 * Grid of P phi samples (P even): phi_j = 2 pi j / P, j < P, and P / 2
 * theta samples theta_i = (i + 1/2) 2 pi / P (no poles), stored row-major
 * [theta][phi] as complex64.  Interpolation maps the samples of a function
 * of degree <= lband on the input grid to its samples on the output grid
 * (exact up to FP32 rounding).  Anterpolation (anterpolate != 0) is the
 * weighted adjoint of the interpolation from the output grid to the input
 * grid, W_out^-1 I^T W_in, with W the quadrature weights (Fejer's first
 * rule in theta times 2 pi / P): the anterpolated samples integrate against
 * every function of degree <= lband as the input samples do.
 *
 * mlfma_fft_plan validates the sizes and prepares a plan on `device`:
 *   lband      band limit (>= 0).
 *   nphi_in, nphi_out  phi counts of the input and output grids: even,
 *              2 lband + 2 <= P <= 1024, no prime factor above 7, and one
 *              item's two LDS regions (2 x 8 x the largest intermediate
 *              array) within 160 KiB (up to P = 120 both ways).
 *   out        receives the plan (owned by the caller; mlfma_fft_destroy).
 * Errors: MLFMA_EINVAL (sizes; no device call is made then), MLFMA_ENOMEM,
 * MLFMA_EDEVICE.
 *
 * mlfma_fft_execute enqueues one kernel on `stream` (a hipStream_t, NULL =
 * null stream) on the plan's device:
 *   in         device, [nitems][nphi_in / 2][nphi_in] complex64.
 *   out        device, [nitems][nphi_out / 2][nphi_out] complex64; must not
 *              overlap `in`.
 *   nitems     number of grids (boxes x right-hand sides); 0 is a no-op.
 * Errors: MLFMA_EINVAL (null plan or buffer, nitems < 0), MLFMA_EDEVICE.
 *
 * mlfma_fft_info: items per workgroup and dynamic LDS bytes of the plan's
 * kernel (host only).  mlfma_fft_destroy: NULL is a no-op.
 */
typedef struct mlfma_fft_s *mlfma_fft_t;
int mlfma_fft_plan(int lband, int nphi_in, int nphi_out, int anterpolate, int device,
                   mlfma_fft_t *out);
int mlfma_fft_execute(mlfma_fft_t plan, const void *in, void *out, int64_t nitems,
                      void *stream);
int mlfma_fft_info(mlfma_fft_t plan, int *items_per_workgroup, int64_t *lds_bytes);
void mlfma_fft_destroy(mlfma_fft_t plan);

/* Host-side queries (no device call). */
int mlfma_tree_info_get(mlfma_tree_t t, mlfma_tree_info *out);
/* perm[s] = caller index of the point at Morton-sorted position s; host [n] */
int mlfma_tree_permutation(mlfma_tree_t t, int64_t *perm);
/* box count (*nbox), integer box coordinates [nbox][3] and parent index
 * [nbox] (-1 at level 1) of level `level` (1..n_levels), in the library's
 * box order; coords and parent may be NULL to query the count only */
int mlfma_tree_level(mlfma_tree_t t, int level, int64_t *nbox,
                     int32_t *coords, int32_t *parent);
/* far-field pairs of level `level` (3..n_levels): observer, source and the
 * offset code (dx+3)*49+(dy+3)*7+(dz+3) of c_obs - c_src; *count receives
 * the pair count; arrays may be NULL to query the count only */
int mlfma_tree_far_list(mlfma_tree_t t, int level, int64_t *count,
                        int32_t *obs, int32_t *src, int32_t *code);
/* near lists of the leaves in CSR form: start [nleaf+1], idx [n_near_pairs] */
int mlfma_tree_near_list(mlfma_tree_t t, int64_t *start, int32_t *idx);
/* info for levels 1..n_levels into out[0..n_levels-1] (max entries given) */
int mlfma_ops_info(mlfma_ops_t ops, mlfma_level_info *out, int max_entries);
/* Device bytes of the handle: *operator_bytes = the translation operator
 * tables of every level (full tables and their antipodal and octant
 * rearrangements, or the sampled tables), *total_bytes = the precompute's
 * planned device bytes (an upper bound of what it allocated; the one
 * mlfma_set_device_memory_limit is checked against).  Host only; either
 * pointer may be NULL. */
int mlfma_ops_memory(mlfma_ops_t ops, int64_t *operator_bytes, int64_t *total_bytes);

/*
 * Diagnostics: copy the spectra the last call left in the workspace.
 *   which 0 = multipole expansions, 1 = local expansions (after L2L)
 *   dst   device buffer of nbox * nrhs * K complex64, layout [box][rhs][K]
 *         with samples [theta][phi], theta ascending, phi_j = 2 pi j / nphi
 */
int mlfma_copy_spectra(mlfma_ops_t ops, int level, int which, int64_t nrhs,
                       void *dst, void *stream);

/*
 * Kernel ids for mlfma_profile_*: one id per kernel of the matvec.
 */
enum mlfma_kernel_id {
    MLFMA_K_GATHER = 0,    /* caller order -> Morton order (+ conj, dtype)   */
    MLFMA_K_P2P = 1,       /* near field                                     */
    MLFMA_K_C2M = 2,       /* leaf signatures                                */
    MLFMA_K_INTERP_S1 = 3, /* M2M: phi DFT on the child grid                 */
    MLFMA_K_INTERP_S2 = 4, /* M2M: per-order theta maps                      */
    MLFMA_K_INTERP_S3 = 5, /* M2M: phi synthesis + shift + aggregation       */
    MLFMA_K_M2L = 6,       /* translation over far lists                     */
    MLFMA_K_ANTERP_S1 = 7, /* L2L: shift + phi DFT on the parent grid        */
    MLFMA_K_ANTERP_S2 = 8, /* L2L: per-order theta maps                      */
    MLFMA_K_ANTERP_S3 = 9, /* L2L: phi synthesis + add                       */
    MLFMA_K_L2O = 10,      /* leaf evaluation + near + scatter               */
    MLFMA_K_INTERP = 11,   /* M2M in one pass (the three maps in LDS)        */
    MLFMA_K_ANTERP = 12,   /* L2L in one pass                                */
    MLFMA_K_COUNT = 13
};

/*
 * Diagnostics: time kernel launches of this handle with HIP events recorded
 * on the launch stream.  Every launch whose id bit is set in kernel_mask is
 * bracketed by an event pair, for at most max_launches launches (the events
 * are created here, or taken from the handle's pool: the events of a
 * session of up to 4096 launches are kept for the next one, so that a
 * session started inside a timed loop after one of the same size creates
 * none; the handle's destruction frees them).  mlfma_profile_end waits for
 * the events, writes the
 * summed milliseconds and launch counts per id into ms[MLFMA_K_COUNT] and
 * launches[MLFMA_K_COUNT], and stops recording.  With MLFMA_PROFILE_SERIAL
 * set in kernel_mask, calls made while recording run every kernel on the
 * caller's stream (as MLFMA_ONE_STREAM does), so that each event pair times
 * its kernel alone rather than while it shares the device with the near
 * field or another level's M2L.
 */
#define MLFMA_PROFILE_SERIAL 0x80000000u
int mlfma_profile_begin(mlfma_ops_t ops, uint32_t kernel_mask,
                        int64_t max_launches);
int mlfma_profile_end(mlfma_ops_t ops, double *ms, int64_t *launches);

/*
 * Diagnostics: the kernel variant the autotuner chose for each level
 * (out[l-1] for levels 1..n_levels; -1 where a level has no such kernel).
 * kernel = MLFMA_K_M2L: 0 per-observer lists from L2, 1 operators staged in
 * LDS, 2 sibling groups, 3 sibling groups with per-source records, 4 the
 * same with a slice-major sweep (for many right-hand sides), 5 the same with
 * parent ranges balanced by record count and parents handed out dynamically,
 * 6 as 5 with a 32-sample operator slice (two workgroups per CU), 7 as 5
 * on antipodal slices (T_{-d}(k) = T_d(-k): the operators of one offset of
 * each +-pair in LDS, two workgroups per CU), 8 as 5 on octant slices (the
 * operators of the offsets (|dx|, |dy|, |dz|) in LDS, reflections as lane
 * permutations); 6, 7 and 8 serve one RHS, calls with several RHS run 5;
 * 9 as 5 on the matrix cores for several RHS (per sample, the parent's
 * children in pairs x four right-hand sides accumulate operator x source
 * over the records on v_mfma_f32_4x4x1f32; at one RHS 3/4 of its tiles
 * are idle, and the precompute timing leaves it out there).  With
 * MLFMA_SAMPLED_OPERATORS only 3, 4, 5 and 9 exist.
 * kernel = MLFMA_K_INTERP or MLFMA_K_ANTERP (entry l = the pair of levels l
 * and l+1, -1 on the leaf level and above level 3): 0 three passes through
 * HBM (ids _S1.._S3), 1 + k one pass with the intermediates in LDS in work
 * split k (children per item, waves per workgroup; 3 splits for the bands
 * 8 -> 13, 2 for 13 -> 20; FP32 only), 4 the fused pair kernel (the maps,
 * shift and sibling sum or add in one launch; bands 8 -> 13 and 13 -> 20,
 * FP32 or BF16x3).
 * kernel = MLFMA_K_P2P (the concurrent schedule; four entries): out[0]
 * where it forks the near field, 1 at the start of the matvec, 2 after C2M,
 * 3 or 4 after the first or second M2M of the upward pass (trees of at least
 * 4 or 5 levels), 0 at the start of the downward pass; out[1] the eighths of
 * the CUs the M2L workgroups of levels above 3 may hold (4, 6, 7 or 8 from
 * the precompute timing); out[2] 1 where the leaf level's M2L runs after the
 * coarser levels' M2L, during the downward pass (trees of more than 3
 * levels), 0 where it runs first, beside the upward pass; out[3] 1 where
 * the near field, forked after an M2M, runs in two halves of its work items,
 * the second forked after the next M2M; all -1 when every kernel runs on the
 * caller's stream.  mlfma_ops_set_variant with this kernel sets the M2L
 * share (level 1, variant 1..8), the leaf M2L order (level 2, variant 0..1),
 * the near-field split (level 3, variant 0..1) or the fork point (any other
 * level, variant 0..4 as the tree allows).
 */
int mlfma_ops_variants(mlfma_ops_t ops, int kernel, int32_t *out, int max_entries);
/* Diagnostics: force a variant of `kernel` on `level` (3..n_levels; for the
 * interpolation ids 3..n_levels-1); used by the tests to check every
 * variant.  EINVAL for an unknown variant, for the one-pass variant where
 * its LDS plan does not fit or MLFMA_BF16X3_INTERP is set, for the pair
 * kernel where the level pair has none, and for M2L forms other than 3, 4,
 * 5 and 9 with MLFMA_SAMPLED_OPERATORS. */
int mlfma_ops_set_variant(mlfma_ops_t ops, int kernel, int level, int variant);

/*
 * Cap on the device bytes mlfma_precompute_operators may allocate (0 = no
 * cap).  The check happens before any device call, so exceeding it returns
 * ENOMEM without touching the GPU.  Process-wide.
 */
void mlfma_set_device_memory_limit(int64_t bytes);

const char *mlfma_status_string(int status);
const char *mlfma_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLFMA_H */
