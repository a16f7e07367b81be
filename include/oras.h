/*
 * oras.h -- C ABI of the MI355X (gfx950) ORAS-FGMRES Helmholtz solver.
 *
 * Solves A u = f for the 3D frequency-domain Helmholtz equation
 * (Delta + k^2) u = f, k = omega / c with c complex in viscous media
 * (arXiv 2110.15113, sec. 2, eq. 1 and eq. 1.1), discretised by the compact
 * lambda-adaptive 27-point finite-difference stencil with PML layers on all
 * faces (sec. 2.3 FDFD; sec. 3.1), by right-preconditioned flexible GMRES
 * (sec. 2.1, sec. 2.2) with the one-level optimized restricted additive
 * Schwarz preconditioner M^{-1} = sum_j R_j^T D_j B_j^{-1} R_j whose local
 * matrices carry Robin (impedance) interface conditions (sec. 2.1), local
 * factorisations computed once at set-up and applied by forward/backward
 * substitution on a whole block of right-hand sides (sec. 2.2, pseudo-block).
 *
 * Conventions (the paper leaves them open; all are fixed here):
 *   time dependence e^{-i omega t}; A = Delta_h + omega^2 M(m~) (paper sign);
 *   attenuation 1/c~ = (1/c)(1 + i/(2Q)); PML s = 1 + i sigma / omega with a
 *   quadratic profile, sigma_max = 3 c_ref ln(1/R0) / (2 L); Robin term
 *   i k S / (s_a h) on the diagonal of B_j per interior face; Boolean
 *   partition of unity (owner computes); stopping test per column
 *   ||b - A x||_2 <= tol ||b||_2 on the FP64 true residual.
 *
 * Memory and layouts
 *   - Every pointer named *_dev is device memory on the context's device,
 *     owned by the caller, and must stay valid until the call returns (all
 *     calls are ordered on the context's stream and synchronise it before
 *     returning).
 *   - Wavefields / right-hand sides: complex128 interleaved (re, im), shape
 *     (nrhs, nz, ny, nx), C order, x fastest -- torch.complex128 contiguous.
 *   - Model arrays (velocity, Q, m): float64, shape (nz, ny, nx).
 *   - Host pointers (*_host, info arrays) are caller-owned host memory.
 *   - The context owns the stencil coefficients, the subdomain factors and
 *     the Krylov workspace; they are freed by oras_destroy.
 *
 * Errors
 *   Every function returns an oras_status and never aborts; oras_last_error()
 *   describes the problem.  Argument and state checks run before any device
 *   call, and model arrays (velocity, Q, m) are checked on the device before
 *   the context changes, so ORAS_E_ARG and ORAS_E_STATE leave the context in
 *   its previous valid state.  A call that fails later (ORAS_E_OOM, ORAS_E_HIP,
 *   ORAS_E_NUMERIC) may have dropped what it was replacing: the operator and
 *   factors for oras_assemble and oras_set_m, the factors for
 *   oras_factor_subdomains, the compressed form for oras_compress_factors.
 *
 * State machine: create -> assemble -> factor_subdomains -> solve ...
 *   assemble and set_m drop the factors (B_j depends on m).
 *   A context is not thread-safe.
 */
#ifndef ORAS_H
#define ORAS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oras_ctx_s* oras_ctx;

typedef enum {
  ORAS_OK = 0,
  ORAS_E_ARG = 1,        /* invalid argument (checked before any device call) */
  ORAS_E_STATE = 2,      /* call out of order, e.g. solve before factor */
  ORAS_E_OOM = 3,        /* device allocation failed or size limit exceeded */
  ORAS_E_HIP = 4,        /* HIP runtime error, or no device in this context */
  ORAS_E_NUMERIC = 5,    /* zero / non-finite pivot, NaN residual, breakdown */
  ORAS_W_NOT_CONVERGED = 100  /* warning: some column hit maxit */
} oras_status;

typedef enum { ORAS_C64 = 1, ORAS_C128 = 2 } oras_prec;

/* Solve flags */
#define ORAS_CONJ 1   /* solve A conj(x) = conj(b), i.e. the adjoint A^H x = b
                         (A is complex symmetric; sec. 2, Method) */
#define ORAS_X0 2     /* x_dev holds an initial guess (warm start / resume) */

typedef struct {
  int nx, ny, nz;      /* nodes per axis, PML included */
  double h;            /* grid step (m) */
  int npml;            /* PML nodes on each face */
  int free_surface;    /* 1: no PML on the top face (k = 0), Dirichlet above */
} oras_grid;

typedef struct {
  double R0;           /* target reflection coefficient (> 0, < 1), e.g. 1e-3 */
  int power;           /* profile exponent, e.g. 2 */
  double c_ref;        /* reference velocity; <= 0 selects the model maximum */
} oras_pml;

/* Interface condition of the subdomain matrices B_j */
typedef enum { ORAS_IFACE_ROBIN = 0, ORAS_IFACE_PML = 1 } oras_iface_kind;

typedef struct {
  int kind;            /* ORAS_IFACE_ROBIN or ORAS_IFACE_PML */
  int power;           /* PML: profile exponent (1..4), e.g. 2 */
  double R0;           /* PML: designed round-trip reflection of the layer, in (0, 1), e.g. 0.3 */
} oras_interface;

typedef struct {
  int restart;         /* FGMRES restart length m (1..200) */
  int maxit;           /* maximum Arnoldi steps per column (>= 1) */
  int flags;           /* ORAS_CONJ | ORAS_X0 */
  int krylov_in_prec;  /* precision of the product A z_j inside the Arnoldi
                          step: 0 = the assembled stencil precision, ORAS_C64
                          (needs a context assembled in ORAS_C64) or ORAS_C128 */
  int z_prec;          /* storage of the preconditioned basis Z: 0 = the factor
                          precision, ORAS_C128, or ORAS_C64 (needs ORAS_C64
                          factors) */
} oras_solve_opts;

typedef struct {
  int* iters;          /* [nrhs] Arnoldi steps taken per column (host, may be NULL) */
  double* rel_res;     /* [nrhs] final true relative residual (host, may be NULL) */
  int* converged;      /* [nrhs] 1 if the column met tol (host, may be NULL) */
  double t_solve;      /* seconds, whole call */
  double t_stencil;    /* seconds in the stencil apply (HIP events) */
  double t_oras;       /* seconds in the ORAS apply */
  double t_ortho;      /* seconds in Gram-Schmidt + Givens */
  int cycles;          /* restart cycles */
  int total_iters;     /* Arnoldi steps of the block */
} oras_solve_info;

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t,
 * NULL = default stream).  device = -1 creates a host-only context that
 * validates arguments but refuses every device operation (ORAS_E_HIP); it
 * exists so argument checking can be tested without a GPU. */
oras_status oras_create(oras_ctx* out, int device, void* hip_stream);

/* Release everything the context owns.  NULL is ignored. */
void oras_destroy(oras_ctx ctx);

/* Message of the last error on this context (never NULL). */
const char* oras_last_error(oras_ctx ctx);

/* The library's own lambda-adaptive weight table (paper sec. 2.3: weights
 * fitted per G = lambda / h by least squares on the phase-velocity
 * dispersion).  Writes up to `capacity` rows of 7 doubles (w1 w2 w3 wm0 wmf
 * wme wmc) into out_host, and the grid G = g0 + dg * row, row < *count.
 * Host only; needs no context.  capacity < count -> ORAS_E_ARG. */
oras_status oras_weight_table(double* out_host, int capacity, double* g0, double* dg, int* count);

/* Assemble the operator (paper eq. 1; sec. 2.3 27-point lambda-adaptive
 * stencil; PML per sec. 3.1).  vel_dev: velocity (m/s, every entry finite and
 * > 0, else ORAS_E_ARG with the number of offending entries);
 * q_dev: quality factor (every entry finite and > 0, same check) or NULL for
 * no attenuation; omega > 0;
 * stencil_prec: ORAS_C128 (all FP64) or ORAS_C64 (the Krylov stencil runs in
 * complex FP32; an FP64 copy is kept for the true residual).  Requires
 * 3 <= nx, ny, nz, 0 <= 2 npml < min(n).  Drops any factors. */
oras_status oras_assemble(oras_ctx ctx, const oras_grid* grid, const double* vel_dev,
                          const double* q_dev, double omega, const oras_pml* pml,
                          int stencil_prec);

/* Replace the real squared slowness m (s^2/m^2, (nz,ny,nx) float64, every
 * entry finite and > 0, else ORAS_E_ARG with the context unchanged) and
 * re-assemble with the stencil weights, PML and Q frozen at the last
 * oras_assemble.  Used by the differentiable forward map.  Drops factors. */
oras_status oras_set_m(oras_ctx ctx, const double* m_dev);

/* Flags of oras_set_m_ex and oras_gradient_ex */
#define ORAS_WEIGHTS_FOLLOW_M 1  /* set_m: recompute the stencil weights from m
                                    (G = 2 pi / (omega h sqrt(m)), sec. 2.3) */
#define ORAS_GRAD_WEIGHTS 1      /* gradient: add the weights' dependence on m */

/* As oras_set_m; with ORAS_WEIGHTS_FOLLOW_M the lambda-adaptive weights are
 * picked again from each node's G at the new m (the attenuation factor and
 * PML stay those of the last oras_assemble).  flags = 0 is oras_set_m. */
oras_status oras_set_m_ex(oras_ctx ctx, const double* m_dev, int flags);

/* Partition the grid into parts[0] x parts[1] x parts[2] cuboids (floor
 * split), extend each by `overlap` layers on interior sides (sec. 2.2:
 * overlapping cuboids), assemble every local matrix B_j with Robin interface
 * faces (sec. 2.1) and factor it on the device (block elimination over the
 * z-planes of the box, explicit inverses of the plane Schur complements by
 * blocked Gauss-Jordan).  factor_prec: ORAS_C64 or ORAS_C128.  Each box must
 * have at least 2 nodes per axis and at most 8192 nodes per z-plane, and
 * overlap must be 0..8.  With 16 subdomains or more, about half of them (a
 * multiple of 8) are factored on a second stream that the context creates at
 * default priority; it is forked from and joined back into the context's
 * stream inside the call.  A zero or non-finite pivot returns ORAS_E_NUMERIC
 * and leaves no factors. */
oras_status oras_factor_subdomains(oras_ctx ctx, const int parts[3], int overlap,
                                   int factor_prec);

/* As oras_factor_subdomains, with the interface condition of B_j chosen by
 * iface (NULL: Robin, as above).  ORAS_IFACE_PML gives PML transmission
 * conditions (sec. 2.2, note on the size of overlap: for finite differences
 * a PML is placed in the overlap region): B_j = R_j A(s_j) R_j^T, the
 * operator assembled with the subdomain's stretching profile and restricted
 * to the box (Dirichlet beyond it).  The profile is the outer PML plus, on
 * each interior side, a layer over the overlap nodes beyond the owned range:
 * sigma = sigma_max (d / L)^power, d the distance from the owned range,
 * L = overlap h, sigma_max = (power + 1) c_ref ln(1 / R0) / (2 L) with the
 * c_ref of the assembly.  PML needs overlap >= 1. */
oras_status oras_factor_subdomains_ex(oras_ctx ctx, const int parts[3], int overlap,
                                      int factor_prec, const oras_interface* iface);

/* Solve A x_c = b_c for nrhs columns with pseudo-block right-preconditioned
 * FGMRES (sec. 2.1, sec. 2.2): FP64 Arnoldi basis, classical Gram-Schmidt,
 * complex Givens, FP64 true residual at each restart.  ORAS runs in the
 * factored precision; by default the product A z_j and the basis Z follow
 * the assembled / factored precisions (all complex64 in mixed mode), and
 * opts->krylov_in_prec / z_prec select complex128 for either (sec. 3: the
 * paper's single-precision runs factor in single precision and keep the
 * Krylov solver in double).  The context must be assembled and factored in
 * the same precision.  b_dev, x_dev: (nrhs,nz,ny,nx) complex128.  tol in
 * (0, 1).  opts NULL = {30, 1000, 0, 0, 0}.  Columns with b = 0 return x = 0
 * (converged).  Returns ORAS_W_NOT_CONVERGED when a column reached maxit,
 * ORAS_E_ARG for an out-of-range option or a precision the context cannot
 * serve. */
oras_status oras_solve(oras_ctx ctx, const void* b_dev, void* x_dev, int nrhs, double tol,
                       const oras_solve_opts* opts, oras_solve_info* info);

/* b_dev (nrhs, nz, ny, nx) complex128 := point sources (sec. 3.1: a delta at
 * a grid node); column c has amplitude (amp_host[2c], amp_host[2c+1]) (1 if
 * amp_host is NULL) at node idx_host[3c..3c+2] = (i, j, k), times the PML
 * factor S there.  Indices must lie inside the grid. */
oras_status oras_point_sources(oras_ctx ctx, const int* idx_host, const double* amp_host,
                               int nrhs, void* b_dev);

/* d_dev (nrhs, nrec) complex128 := u sampled at receivers rec_dev
 * (nrec x 3 int32 (i, j, k), device).  u_dev (nrhs, nz, ny, nx).  This is the
 * observation operator P of the receiver misfit that FWI minimises (sec. 1:
 * the forward engine of frequency-domain FWI; sec. 4: many sources and
 * receivers per frequency).  Receiver indices are copied to the host and
 * checked against the grid first (ORAS_E_ARG). */
oras_status oras_sample(oras_ctx ctx, const void* u_dev, int nrhs, const int* rec_dev, int nrec,
                        void* d_dev);

/* b_dev (nrhs, nz, ny, nx) := P^T d (zero elsewhere, duplicates summed): the
 * adjoint of oras_sample, which carries the data residual back to the grid as
 * the adjoint source of the FWI gradient (sec. 1, sec. 4).  Same receiver
 * layout and checks as oras_sample. */
oras_status oras_spread(oras_ctx ctx, const void* d_dev, int nrhs, const int* rec_dev, int nrec,
                        void* b_dev);

/* g_dev (nz, ny, nx) float64 := -Re sum_c mu_c^H (dA/dm) u_c, the gradient
 * of a real misfit w.r.t. the squared slowness m given the adjoint fields
 * mu (A^H mu = P^T dJ/dd); stencil weights frozen (FWI use, sec. 1, sec. 4). */
oras_status oras_gradient(oras_ctx ctx, const void* u_dev, const void* mu_dev, int nrhs,
                          double* g_dev);

/* As oras_gradient; with ORAS_GRAD_WEIGHTS the gradient also carries the
 * stencil weights' dependence on m (they are picked from the local G, sec.
 * 2.3): -Re sum_k H_k dw_k/dm, H_k = sum_c d(mu_c^H A u_c)/dw_k, dw/dm the
 * weight table's slope times dG/dm = -G / (2 m).  This is the gradient of the
 * map whose weights follow m, so it needs weights that match the current m
 * (after oras_assemble, or oras_set_m_ex with ORAS_WEIGHTS_FOLLOW_M):
 * otherwise ORAS_E_STATE.  Uses scratch of about 7 n doubles. */
oras_status oras_gradient_ex(oras_ctx ctx, const void* u_dev, const void* mu_dev, int nrhs,
                             int flags, double* g_dev);

/* Block low-rank (BLR) plane inverses (sec. 3: the local factors in BLR
 * form with a threshold eps_BLR, 1e-3 in the paper's runs; Table 4).
 *
 * Compresses the current factors in place of the dense plane inverses for
 * every later apply and solve (the factorisation itself is unchanged).  Each
 * plane of a subdomain box is cut into patches of at most pmax x pmax nodes
 * (along x ceil(sx / pmax) parts by floor split, likewise along y; patch
 * index py * npx + px).  Diagonal patch blocks stay dense; every other block
 * is replaced by U V from a cross approximation with complete pivoting that
 * stops once the largest remaining entry is at most eps times the plane's
 * largest entry (so the bound holds for every entry of the error); a block
 * whose rank would exceed b_I b_J / (b_I + b_J) stays dense.  Pivots are
 * chosen in the factor precision.
 *
 * eps in [0, 1), pmax in 2..8 (ORAS_E_ARG otherwise); needs factors
 * (ORAS_E_STATE).  info (host, may be NULL) receives the compression
 * statistics.  The compressed form is dropped by the next assemble, set_m or
 * factor_subdomains.  Device memory: the compressed operands, plus a few
 * bytes per block while compressing; the dense factors stay allocated. */
typedef struct {
  double eps;
  int pmax;
  int max_rank;             /* largest rank of a low-rank block */
  long long blocks;         /* off-diagonal patch blocks, all planes */
  long long lowrank;        /* of which stored as U V */
  double mean_rank;         /* mean rank of the low-rank blocks */
  double stored_entries;    /* complex entries of the compressed inverses */
  double dense_entries;     /* complex entries of the dense inverses (p^2 per plane) */
  double t_compress;        /* wall-clock seconds */
} oras_blr_info;
oras_status oras_compress_factors(oras_ctx ctx, double eps, int pmax, oras_blr_info* info);

/* Test hook: the rank table of plane `plane` of subdomain `sub` after
 * oras_compress_factors, npatch x npatch ints (row I, column J; -1: stored
 * dense, which includes the diagonal) into ranks_host (capacity ints). */
oras_status oras_blr_ranks(oras_ctx ctx, int sub, int plane, int* ranks_host, int capacity,
                           int* npatch);

/* Test hooks running the same kernels as the solver.
 * oras_apply_A: y = A x, the 27-point operator of eq. 1.1 (sec. 2.3), in
 *   precision prec (ORAS_C64 needs stencil_prec C64).
 * oras_apply_M: y = M^{-1} x = sum_j R_j^T D_j B_j^{-1} R_j x, the one-level
 *   ORAS preconditioner of sec. 2.1 with the local solves of sec. 2.2, with
 *   the current factors.
 * x, y: (nrhs, nz, ny, nx) complex128, 1 <= nrhs <= 256, device, caller-owned.
 * Internal staging buffers are allocated by the context and kept. */
oras_status oras_apply_A(oras_ctx ctx, const void* x_dev, void* y_dev, int nrhs, int prec);
oras_status oras_apply_M(oras_ctx ctx, const void* x_dev, void* y_dev, int nrhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): oras_apply_A
 * with no allocation.  Same arguments, checks, kernels and results as
 * oras_apply_A (y_dev is written with y = A x, bitwise equal to it); the
 * staging it needs (x and y in the internal layout, and x rounded to complex64
 * for ORAS_C64: 16 + 16 (+ 8) bytes per node and padded right-hand side,
 * right-hand sides padded to a multiple of 8) lives in a fixed device array of
 * oras_noalloc_scratch_bytes() bytes (64 MiB) that every GPU the library runs
 * on holds until the process ends.  A larger request returns ORAS_E_ARG before
 * any device work.  All calls on one GPU share that GPU's array, so calls that
 * overlap on one GPU (several streams or host threads) race; calls ordered on
 * one stream do not. */
oras_status oras_apply_A_noalloc(oras_ctx ctx, const void* x_dev, void* y_dev, int nrhs, int prec);
/* Size in bytes of the fixed staging array of oras_apply_A_noalloc. */
size_t oras_noalloc_scratch_bytes(void);

/* Pivot statistics of the last oras_factor_subdomains (sec. 2.2: the local
 * matrices are factorised once at set-up).  The plane Schur complements S_k
 * are inverted without row exchanges, so the smallest pivot relative to the
 * plane's largest entry,
 *     r = min |pivot of S_k| / max |entry of S_k|,
 * measures how close each elimination came to breaking down (a zero or
 * non-finite pivot already fails the factorisation with ORAS_E_NUMERIC).
 * min_ratio receives the smallest r over all subdomain planes, sub and plane
 * where it occurs; ratios_host (capacity doubles, may be NULL) receives r for
 * every subdomain plane at index sub * max_planes + plane (NaN beyond a box's
 * planes), *max_planes its second dimension.  Any output may be NULL.
 * ORAS_E_STATE without factors, ORAS_E_ARG if capacity is too small. */
oras_status oras_factor_stats(oras_ctx ctx, double* min_ratio, int* sub, int* plane,
                              double* ratios_host, int capacity, int* max_planes);

/* Wall-clock seconds of the last oras_assemble and of the last
 * oras_factor_subdomains (the paper's set-up time T_f, sec. 3.2). */
oras_status oras_timings(oras_ctx ctx, double* t_assemble, double* t_factor);

/* Per-launch timing of the plane GEMM of the ORAS apply (the local
 * forward/backward substitutions, sec. 2.2).  enable != 0 records a HIP
 * event pair around every plane product on the context stream (the apply
 * then synchronises once to read them) and resets the counters. */
oras_status oras_profile(oras_ctx ctx, int enable);

/* Accumulated plane-GEMM time (s), number of plane products, and their
 * algorithmic work: 8 p^2 nrhs flops and p^2 + 2 p nrhs (+ p nrhs backward)
 * complex entries moved per subdomain, p = plane size of its box.  With BLR
 * inverses a plane product is the projection and expansion pair, and the
 * work is that of the stored blocks: 8 nrhs flops per stored entry, the
 * stored entries plus the gathered and written rows. */
oras_status oras_kernel_stats(oras_ctx ctx, double* gemm_seconds, long long* gemm_launches,
                              double* gemm_flops, double* gemm_bytes);

/* Accumulated time (s) and algorithmic bytes of the plane right-hand-side
 * kernels, which carry the restriction R_j v of the ORAS apply (sec. 2.1)
 * fused with the block couplings of the plane recursion (sec. 2.2), under
 * the same oras_profile switch: per active subdomain plane of p nodes,
 * p nrhs (16 (v, forward only) + b (neighbouring plane of y, except on the
 * first forward plane) + t written) + 9 p b bytes of couplings, b the factor
 * precision's bytes per complex value and t written as six bf16 pieces (12
 * bytes) for the complex-FP32 dense products, else one value.  Each time is
 * measured from the end of the previous plane step (or from the start of the
 * apply) to the end of the kernel, so it includes one launch gap. */
oras_status oras_rhs_stats(oras_ctx ctx, double* seconds, double* bytes);

/* Copy the 27 FP64 stencil coefficients per node, layout (27, nz, ny, nx)
 * complex128, slot e = (ez+1)*9 + (ey+1)*3 + (ex+1). */
oras_status oras_coefficients(oras_ctx ctx, void* out_dev);

/* Number of subdomains and the box / owned cuboid of subdomain j
 * (lo x,y,z, hi x,y,z, olo..., ohi...) into box12_host. */
oras_status oras_subdomain(oras_ctx ctx, int j, int* nsub, int* box12_host);

#ifdef __cplusplus
}
#endif
#endif
