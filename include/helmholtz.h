/*
 * helmholtz.h - C ABI of the MI355X (gfx950) Helmholtz multigrid library.
 *
 * The library solves H x = b for the pressure-correction (Helmholtz) operator
 * of a semi-implicit atmospheric model on a cubed-sphere mesh of vertical
 * columns, preconditioned by the tensor-product multigrid V-cycle of
 * Maynard, Melvin and Mueller (Section 3.6 of their paper): block-Jacobi
 * smoothing with exact tridiagonal solves in each column (Eq. jacobi),
 * horizontal-only 2x2 coarsening, prolongation by natural injection,
 * restriction as its dual, and a few smoothing sweeps instead of a coarse
 * solve (Algorithm 1). The Krylov loop is conjugate gradients or BiCGStab
 * (Section 4.1).
 *
 * Operator. H is a symmetric positive definite face-coupling operator that
 * stands in for the paper's finite-element H (Eq. helmholtz_operator):
 *   (H x)[k,c] = delta[k,c] x[k,c]
 *              + sum over the 4 horizontal faces f of c: K_h(f,k) (x[k,c] - x[k,nbr_f(c)])
 *              + kv[k,c]   (x[k,c] - x[k+1,c])   (k < nz-1)
 *              + kv[k-1,c] (x[k,c] - x[k-1,c])   (k > 0).
 * Coarse operators are re-discretised (Section 3.6, scalings of Eq. DH_ratios):
 * a coarse horizontal face takes the mean of its two fine faces, the coarse
 * kv and delta the sum over the four children.
 *
 * Mesh. C<N>: 6 panels of N x N columns, column index c = p*N*N + j*N + i.
 * Directions E=0 (+i), W=1, N=2 (+j), S=3. Panel orientation (normal, E axis,
 * N axis) on the cube: p0 (+x,+y,+z), p1 (+y,-x,+z), p2 (-x,-z,-y),
 * p3 (-y,-z,+x), p4 (+z,-x,-y), p5 (-z,+y,+x). Each horizontal face is stored
 * once, as the E face (slot 0) or the N face (slot 1) of one of its cells.
 * Level l = 1..L has N / 2^(l-1) columns per panel edge; coarse column of
 * (p,i,j) is (p,i/2,j/2).
 *
 * Layouts. Coefficients: kh[2][nz][ncol], kv[nz-1][ncol], delta[nz][ncol].
 * Vectors: [batch][nz][ncol], contiguous, column index fastest, float64
 * unless the name says f32. All array pointers are DEVICE pointers unless
 * marked "host". Every call is ordered on the given HIP stream.
 *
 * Memory. The library never allocates device memory: the caller passes one
 * workspace of helmholtz_workspace_bytes(cfg) bytes to helmholtz_create and
 * keeps it alive until helmholtz_destroy. The handle itself lives in host
 * memory (plus a small pinned host buffer for the solver's scalars). The one
 * exception is a static device array of HELMHOLTZ_NOALLOC_SCRATCH_BYTES per
 * GPU, loaded with the library, that only helmholtz_vcycle_noalloc uses.
 * Calls on one handle must not overlap (a handle is not thread-safe and its
 * workspace is shared by all its calls).
 *
 * Errors. Functions return HELMHOLTZ_OK (0) or a negative code;
 * helmholtz_solve may also return HELMHOLTZ_NOT_CONVERGED (1), in which case
 * its outputs are still valid. helmholtz_strerror(code) names the code.
 */
#ifndef HELMHOLTZ_H
#define HELMHOLTZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct helmholtz_s* helmholtz_t;
typedef struct ihipStream_t* helmholtz_stream_t; /* a hipStream_t; NULL = default stream */

enum {
    HELMHOLTZ_OK = 0,
    HELMHOLTZ_NOT_CONVERGED = 1, /* solve hit maxiter; outputs valid              */
    HELMHOLTZ_EINVAL = -1,       /* bad argument, config or coefficient value      */
    HELMHOLTZ_ESHAPE = -2,       /* N % 2^(L-1) != 0, nz > HELMHOLTZ_NZ_MAX, batch
                                    > max_batch, or sizes beyond 32-bit indexing   */
    HELMHOLTZ_EWORKSPACE = -3,   /* workspace NULL, too small or misaligned        */
    HELMHOLTZ_ENONFINITE = -4,   /* NaN/Inf in coefficients or in a solve          */
    HELMHOLTZ_EHIP = -5,         /* a HIP runtime call or kernel launch failed     */
    HELMHOLTZ_ESCRATCH = -6      /* helmholtz_vcycle_noalloc: the level vectors do
                                    not fit HELMHOLTZ_NOALLOC_SCRATCH_BYTES          */
};

enum { HELMHOLTZ_FP64 = 0, HELMHOLTZ_FP32 = 1 };               /* V-cycle precision   */
/* Krylov method of helmholtz_solve (Section 4.1): conjugate gradients with the
 * Fletcher-Reeves (standard) or Polak-Ribiere (flexible) beta, or BiCGStab. */
enum { HELMHOLTZ_CG_STANDARD = 0, HELMHOLTZ_CG_FLEXIBLE = 1, HELMHOLTZ_BICGSTAB = 2 };

#define HELMHOLTZ_NZ_MAX 120
#define HELMHOLTZ_WORKSPACE_ALIGN 256

typedef struct {
    int32_t N;            /* columns per panel edge on the finest level, >= 1             */
    int32_t nz;           /* vertical levels, 1 .. HELMHOLTZ_NZ_MAX                         */
    int32_t nlevels;      /* multigrid levels L >= 1; N must be divisible by 2^(L-1)        */
    int32_t n_pre;        /* pre-smoothing sweeps (>= 0), Algorithm 1                        */
    int32_t n_post;       /* post-smoothing sweeps (>= 0)                                    */
    int32_t n_coarse;     /* sweeps on the coarsest level (>= 1)                             */
    double omega;         /* over-relaxation of Eq. jacobi, 0 < omega <= 1.5                 */
    int32_t mg_precision; /* HELMHOLTZ_FP64 or HELMHOLTZ_FP32 (V-cycle arithmetic)           */
    int32_t cg_variant;   /* HELMHOLTZ_CG_STANDARD, _CG_FLEXIBLE or HELMHOLTZ_BICGSTAB       */
    int32_t max_batch;    /* largest batch any call will pass, >= 1                          */
    int32_t stencil;      /* 7 (or 0): nearest vertical couplings only; 9: also couplings two
                             levels apart (Section 3.5), created with helmholtz_create9     */
    int32_t weighted;     /* 0: symmetric H; 1: row-weighted, non-symmetric H = delta + S L,
                             created with helmholtz_create_weighted (needs
                             HELMHOLTZ_BICGSTAB and the 7-point stencil)                    */
} helmholtz_config;

/* Bytes of device workspace that helmholtz_create needs for cfg; 0 if cfg is
 * invalid. Pure host function, no HIP calls. */
size_t helmholtz_workspace_bytes(const helmholtz_config* cfg);

/* Build the operator hierarchy (Section 3.6): mesh tables of every level,
 * coarse coefficients by re-discretisation, the column factorisations used by
 * the smoother (the LU factors of the column operator that the block-Jacobi
 * step needs) and float32 copies of all of them.
 *   kh    [2][nz][ncol] coupling across each column's E (slot 0) and N (slot 1) face, >= 0
 *   kv    [nz-1][ncol]  coupling between levels k and k+1 (may be NULL if nz == 1), >= 0
 *   delta [nz][ncol]    zero-order term, > 0
 *   workspace           device buffer of >= helmholtz_workspace_bytes(cfg) bytes,
 *                       HELMHOLTZ_WORKSPACE_ALIGN-aligned, owned by the caller
 * The coefficients are copied; the caller may free them when this returns.
 * Synchronises `stream` once. On success *out holds a new handle. */
int helmholtz_create(const helmholtz_config* cfg, const double* kh, const double* kv,
                     const double* delta, void* workspace, size_t workspace_bytes,
                     helmholtz_stream_t stream, helmholtz_t* out);

/* The 9-cell stencil of Section 3.5: H also couples each cell to the cells two
 * levels above and below,
 *   (H x)[k,c] += kv2[k,c] (x[k,c] - x[k+2,c])   (k < nz-2)
 *              + kv2[k-2,c] (x[k,c] - x[k-2,c])  (k > 1),
 * and the smoother's column matrix drops those couplings but keeps their
 * contribution to the diagonal (Section 3.6: the block-tridiagonal Hz of the
 * block-Jacobi step), so a sweep no longer solves a column exactly. Coarse
 * levels sum kv2 over the four children, like kv.
 *   kv2   [nz-2][ncol]  >= 0 (may be NULL if nz <= 2)
 * cfg->stencil must be 9; the other arguments are those of helmholtz_create,
 * which rejects stencil 9. */
int helmholtz_create9(const helmholtz_config* cfg, const double* kh, const double* kv,
                      const double* kv2, const double* delta, void* workspace,
                      size_t workspace_bytes, helmholtz_stream_t stream, helmholtz_t* out);

/* The non-symmetric operator of Section 5.1: the paper's horizontal term acts
 * like -(1/rho*) div(rho* theta* grad), a symmetric face-weighted Laplacian
 * scaled row by row (Eq. continuum_pressure_operator). With a row weight s
 * (the role of 1/rho*):
 *   (H x)[k,c] = delta[k,c] x[k,c] + s[k,c] (L x)[k,c],   L x = the flux terms
 * of helmholtz_create's operator, so the two cells of a face see different
 * couplings and CG does not apply (cfg->cg_variant must be HELMHOLTZ_BICGSTAB,
 * cfg->weighted 1, stencil 7). The column matrix of the smoother is the
 * column part of H (rows weighted the same way); coarse levels take the mean
 * of the four children's s. The adjoint calls below use H^T = delta + L S
 * with the transposed V-cycle (the transpose of the V-cycle of H).
 *   s     [nz][ncol]   > 0
 * Other arguments as for helmholtz_create. */
int helmholtz_create_weighted(const helmholtz_config* cfg, const double* kh, const double* kv,
                              const double* delta, const double* s, void* workspace,
                              size_t workspace_bytes, helmholtz_stream_t stream,
                              helmholtz_t* out);

/* Replace the operator of an existing handle: the coefficient part of
 * set-up only (coarse levels by re-discretisation, column factors, float32
 * copies); the mesh tables and the workspace stay. Arguments as for the
 * create call that made the handle: kv2 non-NULL exactly for a 9-cell handle
 * with nz > 2, s exactly for a weighted one. Validation as at create; on an
 * error the handle holds no usable operator until an update succeeds.
 * Synchronises `stream` once. */
int helmholtz_update(helmholtz_t h, const double* kh, const double* kv, const double* kv2,
                     const double* delta, const double* s, helmholtz_stream_t stream);

/* Release host state (handle, pinned scalars). Never touches the workspace. */
int helmholtz_destroy(helmholtz_t h);

/* y = H x on the finest level (the operator of Eq. helmholtz), float64,
 * x and y [batch][nz][ncol], must not overlap. Asynchronous. */
int helmholtz_apply(helmholtz_t h, const double* x, double* y, int32_t batch,
                    helmholtz_stream_t stream);

/* x = M b: one V-cycle of Algorithm 1 from a zero initial guess, in the
 * handle's mg_precision (float32 V-cycles round b once and widen x once).
 * This is also the preconditioner-only solver PreOnly(H, M) of Section 4.1:
 * with nlevels = 1 it is the line relaxation P_H^(Jac)(omega, n_coarse),
 * n_coarse block-Jacobi sweeps (Eq. jacobi) from x = 0.
 * b and x [batch][nz][ncol] float64, must not overlap. Asynchronous. */
int helmholtz_vcycle(helmholtz_t h, const double* b, double* x, int32_t batch,
                     helmholtz_stream_t stream);

/* helmholtz_vcycle for callers that cannot allocate device memory at call
 * time (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same V-cycle, with the same kernels and the same
 * result bit for bit, but its level vectors (right-hand side, iterate and
 * Jacobi partner of every level, 3 * batch * nz * ncol_l values of the
 * handle's mg_precision per level l, columns padded to multiples of 32) live
 * in a static device array of HELMHOLTZ_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends, instead of in
 * the workspace. The call allocates and frees nothing (with the kernel
 * timing hook off it creates no HIP objects either). Nothing in the scratch
 * needs to start at zero; it keeps the last call's contents. Every call on
 * one GPU shares that GPU's array, so calls that overlap on one GPU (any
 * handle, any stream) race and must be serialised by the caller.
 * The calling thread's current device must be the one the handle was created
 * on (else HELMHOLTZ_EINVAL). Returns HELMHOLTZ_ESCRATCH, launching nothing,
 * when the level vectors exceed the array: e.g. C96 x 30 with 5 levels fits
 * at batch 1 in float64 and at batch 2 in float32, C192 x 70 does not.
 * b and x [batch][nz][ncol] float64, must not overlap. Asynchronous. */
#define HELMHOLTZ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int helmholtz_vcycle_noalloc(helmholtz_t h, const double* b, double* x, int32_t batch,
                             helmholtz_stream_t stream);

/* Same V-cycle entirely in float32 (coefficients, vectors and accumulation).
 * b and x [batch][nz][ncol] float32, must not overlap. Asynchronous. */
int helmholtz_vcycle_f32(helmholtz_t h, const float* b, float* x, int32_t batch,
                         helmholtz_stream_t stream);

/* Solve H x = b by a Krylov method of Section 4.1 preconditioned by one
 * V-cycle per preconditioner application, from x = 0, independently for each
 * right-hand side. cg_variant selects conjugate gradients (one product with H
 * and one V-cycle per iteration) or right-preconditioned BiCGStab (two of
 * each per iteration, shadow residual b; a zero inner product before
 * convergence stops that right-hand side and the call returns
 * HELMHOLTZ_NOT_CONVERGED). The outer loop (residual update, dot products,
 * norms, solution update) is float64; the V-cycle runs in mg_precision.
 *   rtol     stop when ||r||_2 <= rtol ||b||_2 (recursively updated residual)
 *   maxiter  largest number of iterations, >= 1
 *   iters    host [batch]: iterations taken per right-hand side (may be NULL)
 *   relres   host [batch]: final ||r||_2 / ||b||_2 (0 when b = 0) (may be NULL)
 * Synchronises `stream` once per iteration for the convergence test.
 * Returns HELMHOLTZ_NOT_CONVERGED if any right-hand side hit maxiter and
 * HELMHOLTZ_ENONFINITE if b or a residual norm is not finite. */
int helmholtz_solve(helmholtz_t h, const double* b, double* x, int32_t batch, double rtol,
                    int32_t maxiter, int32_t* iters, double* relres,
                    helmholtz_stream_t stream);

/* Gradients of L = sum_b g_b . x_b with respect to the operator's
 * coefficients, given x = H^-1 b and the adjoint lam = H^-1 g (H is
 * symmetric, so the adjoint solve is helmholtz_solve on g):
 *   g_kh[s][k][c] = -sum_b (lam[k,c]-lam[k,n]) (x[k,c]-x[k,n]), n the E (s=0) or N (s=1) neighbour
 *   g_kv[k][c]    = -sum_b (lam[k,c]-lam[k+1,c]) (x[k,c]-x[k+1,c])
 *   g_delta[k][c] = -sum_b lam[k,c] x[k,c]
 * lam, x [batch][nz][ncol]; outputs are overwritten (g_kv may be NULL if nz == 1).
 * Asynchronous. */
int helmholtz_face_grad(helmholtz_t h, const double* lam, const double* x, int32_t batch,
                        double* g_kh, double* g_kv, double* g_delta, helmholtz_stream_t stream);

/* helmholtz_face_grad for a 9-cell handle, adding g_kv2 [nz-2][ncol] (the
 * same flux-form rule on the faces k | k+2, summed over the batch; may be NULL
 * to skip it, must be NULL for a 7-point handle). */
int helmholtz_face_grad9(helmholtz_t h, const double* lam, const double* x, int32_t batch,
                         double* g_kh, double* g_kv, double* g_kv2, double* g_delta,
                         helmholtz_stream_t stream);

/* Adjoint counterparts, for the gradient of a loss of x = H^-1 b: y = H^T x;
 * one V-cycle of the transposed hierarchy; the solve of H^T lam = g (same
 * Krylov method and preconditioner settings as helmholtz_solve). On a
 * symmetric handle they are helmholtz_apply / _vcycle / _solve. Arguments,
 * layouts and stream behaviour as for those calls. */
int helmholtz_apply_adjoint(helmholtz_t h, const double* x, double* y, int32_t batch,
                            helmholtz_stream_t stream);
int helmholtz_vcycle_adjoint(helmholtz_t h, const double* b, double* x, int32_t batch,
                             helmholtz_stream_t stream);
int helmholtz_solve_adjoint(helmholtz_t h, const double* g, double* lam, int32_t batch,
                            double rtol, int32_t maxiter, int32_t* iters, double* relres,
                            helmholtz_stream_t stream);

/* Coefficient gradients of L = g . x for a weighted handle, given
 * lam = H^-T g and x, summed over the batch (dH/dK = S a a^T for a face
 * vector a = e_i - e_j):
 *   g_kh[s][k][c] = -sum_b (s lam[k,c] - s lam[k,n]) (x[k,c] - x[k,n]), n the E/N neighbour
 *   g_kv[k][c]    = -sum_b (s lam[k,c] - s lam[k+1,c]) (x[k,c] - x[k+1,c])
 *   g_delta       = -sum_b lam x,   g_s = -sum_b lam (L x)
 * (each s at the cell of the lam it multiplies). Output layouts as for
 * helmholtz_face_grad, g_s [nz][ncol]; all overwritten. Asynchronous. */
int helmholtz_face_grad_weighted(helmholtz_t h, const double* lam, const double* x,
                                 int32_t batch, double* g_kh, double* g_kv, double* g_delta,
                                 double* g_s, helmholtz_stream_t stream);

/* Mesh tables of C<N> as built by the library (host arrays, int32):
 *   nbr    [4][6N^2]  neighbour column in directions E, W, N, S
 *   ftab   [4][6N^2]  stored face of each direction: slot*ncol + owner column
 *   parent [6N^2]     column of C<N/2> that contains each column (NULL, or ignored if N is odd)
 * Pure host function. */
int helmholtz_mesh_tables(int32_t N, int32_t* nbr, int32_t* ftab, int32_t* parent);

/* Kernel timing (instrumentation, not part of the method). While enabled,
 * every launch of the profiled kernels is bracketed by HIP events on the
 * stream it runs on; helmholtz_profile_read waits for the recorded events
 * and returns the accumulated device time, the number of launches and the
 * algorithmic bytes those launches had to move (the words each unknown must
 * read and write, times the unknowns processed). Enabling resets the counts.
 * Profiled kernels:
 *   HELMHOLTZ_PROF_SWEEP_FINE   block-Jacobi sweep on the finest level
 *                               (plain mode: reads b, x, two face couplings
 *                               and the two column factors, writes x_new:
 *                               7 words per unknown)
 *   HELMHOLTZ_PROF_APPLY_FINE   float64 operator apply on the finest level
 *                               (reads x, kh[2], kv, delta, writes y: 6 words)
 *   HELMHOLTZ_PROF_VCYCLE       each whole V-cycle inside helmholtz_solve (one
 *                               event pair around all its launches, gaps
 *                               between them included); bytes: the words its
 *                               kernels must move on every level (first sweep
 *                               from zero 4, further sweeps 7, residual +
 *                               restriction 6.25, sweep with prolongation
 *                               7.25; one more per sweep and residual for the
 *                               9-cell and the row-weighted operator), times
 *                               the unknowns of the level and the batch */
enum { HELMHOLTZ_PROF_SWEEP_FINE = 0, HELMHOLTZ_PROF_APPLY_FINE = 1, HELMHOLTZ_PROF_VCYCLE = 2,
       HELMHOLTZ_PROF_COUNT = 3 };
int helmholtz_profile_enable(helmholtz_t h, int enable);
int helmholtz_profile_read(helmholtz_t h, int32_t kernel, double* ms /* host */,
                           int64_t* launches /* host */, double* bytes /* host */);

/* Achievable-bandwidth yardstick (instrumentation, not part of the method):
 * one launch of a plain streaming kernel over n float32 values, 16-byte
 * vector accesses, one pass:
 *   HELMHOLTZ_BW_READ   reads a; writes one partial sum per 4096 values to c
 *                       (so c needs n / 4096 floats rounded up)
 *   HELMHOLTZ_BW_WRITE  c = s
 *   HELMHOLTZ_BW_COPY   c = a
 *   HELMHOLTZ_BW_TRIAD  c = a + s b
 * a, b, c device arrays (unused ones may be NULL), 16-byte aligned, n a
 * multiple of 4, n / 4096 < 2^31. Asynchronous. */
enum { HELMHOLTZ_BW_READ = 0, HELMHOLTZ_BW_WRITE = 1, HELMHOLTZ_BW_COPY = 2,
       HELMHOLTZ_BW_TRIAD = 3 };
int helmholtz_bandwidth_kernel(int32_t kind, const float* a, const float* b, float* c, int64_t n,
                               float s, helmholtz_stream_t stream);

/* Static description of a return code. */
const char* helmholtz_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* HELMHOLTZ_H */
