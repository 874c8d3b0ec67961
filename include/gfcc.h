/*
 * gfcc.h -- C ABI of the MI355X IP-GFCCSD linear-solve library (libgfcc.so).
 *
 * Operation (arXiv 2010.04768, Theory section): for orbitals p, q (occupied or
 * virtual; the benchmarks use occupied ones) and real frequencies omega, the retarded ionisation (IP) term of the coupled-cluster
 * Green's function in the GFCCSD truncation,
 *
 *     G_qp(omega) = c_q^T X_p(omega),   (omega + Hbar_N - i*eta) X_p = b_p,
 *
 * (the linear system for X_p and the compact form of G; the bilinear product
 * c^T X of the model-order-reduction equations), where
 *   Hbar_N  = connected similarity-transformed Hamiltonian e^-T H e^T - E0,
 *             restricted to the 1h + 2h1p space of X_p (the X_p expansion),
 *   b_p     = abar_p |Phi>  (= the 1h unit vector e_p for occupied p; for virtual
 *             p = o + a it is [a_a, T]|Phi>: t_i^a on 1h, t_ij^ab on 2h1p),
 *   c_q     = <Phi|(1 + Lambda) abar_q^+ restricted to the same space (for
 *             virtual q = o + a: l_i^a on 1h, 2 l_kl^ac - l_kl^ca on 2h1p),
 * with T and Lambda truncated at singles and doubles.  The systems are solved
 * by restarted GMRES (GFCC Workflow and Bottlenecks section), optionally right-preconditioned.
 *
 * Closed-shell spin-adapted basis, dimension D = o + o*o*v:
 *     x[0 .. o)                     = r_i     (1h)
 *     x[o + (i*o + j)*v + a]        = r_ija   (2h1p, the i(alpha) j(beta) -> a(beta) amplitude)
 * Complex vectors at this boundary are interleaved (re, im) FP64 pairs,
 * i.e. a complex vector of dimension D is 2*D doubles.
 *
 * Conventions for every entry point:
 *   - All array pointers are DEVICE pointers unless the comment says "host".
 *   - Row-major, 64-bit dimensions.  Orbitals are ordered occupied first.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Entry points return after enqueueing unless stated "blocking".
 *   - Nothing throws across the ABI; every function returns a gfcc_status.
 *     On failure gfcc_last_error() returns a thread-local message.
 *   - Input arrays are borrowed for the duration of the call only, except the
 *     amplitudes t2 and l2 of gfcc_system (borrowed until gfcc_destroy).
 *     Output arrays are owned by the caller.
 */
#ifndef GFCC_H
#define GFCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gfcc_ctx gfcc_ctx; /* opaque: owns intermediates and workspaces */

typedef enum {
  GFCC_OK = 0,
  GFCC_E_ARG = -1,    /* bad argument or dimension */
  GFCC_E_OOM = -2,    /* device allocation failed */
  GFCC_E_HIP = -3,    /* HIP runtime error */
  GFCC_E_STATE = -4,  /* call not valid in the context's state */
  GFCC_W_NOCONV = 1   /* solve finished; some right-hand sides did not converge (see info) */
} gfcc_status;

/* Arithmetic of the sigma product.  The FP32/BF16/FP16 forms run the two-body
 * (W-tensor) contractions on MFMA in that precision with FP32 accumulation;
 * one-body terms, Arnoldi, Givens and the true residual stay FP64 and the
 * solver refines iteratively in FP64 (GMRES-IR).  Operands get power-of-two scales
 * (amax -> [1, 2)): per tensor for the intermediates, and for FP16, whose exponent
 * range is narrow, per sigma call for the vectors, computed on the GPU. */
typedef enum { GFCC_FP64 = 0, GFCC_FP32_IR = 1, GFCC_BF16_IR = 2, GFCC_FP16_IR = 3 } gfcc_precision;

typedef enum {
  GFCC_PC_NONE = 0,   /* plain GMRES */
  GFCC_PC_JACOBI = 1, /* right preconditioner 1/(omega - i eta + diag(Hbar_N)) (Workflow section) */
  GFCC_PC_MLP = 2     /* learned residual->correction network, flexible GMRES; Jacobi fallback */
} gfcc_precond;

/* One closed-shell system.  Device pointers, FP64.
 *   eps [n]            orbital energies (Fock matrix diag(eps)), occupied first
 *   L   [Q][n][n]      Cholesky vectors, symmetric in (p,q):
 *                      (pq|rs) = sum_Q L[Q][p][q] L[Q][r][s]   (Implementation Details: Cholesky ERIs)
 *   t1  [o][v], t2 [o][o][v][v]   ground-state amplitudes t_i^a, t_ij^ab, with the
 *                      closed-shell pair symmetry t2[i][j][a][b] = t2[j][i][b][a]
 *   l1, l2             Lambda amplitudes in the same layout (l2 with the same pair
 *                      symmetry); NULL means Lambda = T^dagger (l1 = t1, l2 = t2).
 * Ownership: eps, L, t1 and l1 are read during gfcc_build_intermediates only.
 * t2, and l2 when it differs from t2, are BORROWED by the context: the sigma
 * product and the virtual-orbital vectors read them in place (at the C60-shaped
 * 120/600/3000 system t2 alone is 41.5 GB), so they must stay valid and unchanged
 * until gfcc_destroy.                                                        */
typedef struct {
  int64_t n_occ, n_vir, n_chol;
  const double* eps;
  const double* L;
  const double* t1;
  const double* t2;
  const double* l1;
  const double* l2;
} gfcc_system;

/* Build the per-system intermediates (blocks of Hbar_N, its exact diagonal,
 * the left vectors c_q for all occupied q; reduced-precision copies follow on
 * first use) on the GPU; the paper precomputes these constant intermediates
 * before the GFCC loop (Implementation Details).  The context copies t1 and l1
 * and borrows t2 (and l2 when its contents differ from t2), see gfcc_system.
 * Nothing of size o^2 v^2 is stored besides the ring matrix [Wovvo | Wovov]
 * (2 (ov)^2 doubles); the build's own temporaries are chunked to the free device
 * memory (gfcc_plan_memory gives the budget).  With the environment variable
 * GFCC_VERBOSE set the byte budget per operand is printed to stderr before
 * allocating.  Blocking.  *out receives a new context (free it with
 * gfcc_destroy).  Errors: E_ARG for bad dimensions or null pointers, E_OOM when
 * device memory runs out. */
gfcc_status gfcc_build_intermediates(const gfcc_system* sys, void* stream, gfcc_ctx** out);

/* Build the context of the advanced, electron-attached (EA) term of the same system
 * (Theory section: the second term of the Green's function, the Y_q expansion in
 * one-particle and two-particle-one-hole operators and its linear system):
 *
 *     G^EA_pq(omega) = c'_p^T Y_q(omega),   (omega - Hbar_N + i*eta) Y_q = b'_q,
 *     b'_q = abar_q^+ |Phi>,   c'_p = <Phi|(1 + Lambda) abar_p   (on 1p + 2p1h).
 *
 * Closed-shell spin-adapted basis (doublet), dimension D = v + o*v*v:
 *     y[0 .. v)                  = y_a     (coefficient of a^+_{a alpha})
 *     y[v + (j*v + a)*v + b]     = y_jab   (coefficient of a^+_{a alpha} a^+_{b beta} a_{j beta})
 * the same-spin component being y_jab - y_jba.
 *
 * The returned context works with these entry points, with these meanings:
 *   gfcc_dims        D = v + o v^2
 *   gfcc_sigma       Y = Hbar_N X on 1p + 2p1h, GFCC_FP64 or GFCC_FP16_IR (FP16 copies of the
 *                    five two-body blocks and t2 with power-of-two scales, FP32 accumulation, the
 *                    vector scale taken on the GPU per call); E_ARG for FP32 and BF16
 *   gfcc_solve_batch for right-hand side r: Y_{p[r]} at omega[r] (the system above, solved as
 *                    (-omega - i eta + Hbar_N) Y = -b' by the same GMRES; Jacobi uses the EA
 *                    diagonal); G[r][k] = c'_{q[k]} . Y_{p[r]} = G^EA_{q[k] p[r]}; X receives Y.
 *                    GFCC_FP64 or GFCC_FP16_IR (FP16 sigma in the restart cycles, FP64 true
 *                    residuals between them); GFCC_PC_MLP is E_STATE.
 *   gfcc_solve_shifts multi-shift GMRES over all frequencies of each right-hand side orbital, the same
 *                    G^EA_{q p}(omega) layout (FP64; a fallback runs in FP64 or FP16-IR without the
 *                    network)
 *   gfcc_greens, gfcc_greens_noalloc   G[r][k] = c'_{q[k]} . X[r]
 *   gfcc_export      FOO, FVV, FOV (the one-body blocks shared with the IP term) and DIAG [D]
 *   gfcc_prof_*, gfcc_destroy
 * Every other entry point returns E_STATE on it.  The full retarded function is
 * G_pq = G^IP_pq + G^EA_pq (the IP context's G[r][k] is G^IP_{p[r] q[k]}).
 *
 * Storage (FP64): the particle-particle ladder Wvvvv as a [v^2][v^2] matrix (the sigma
 * product's dominant operand, 2 o v^4 flops per vector), Wvvvo [o v^2][v], the 1p rows
 * [v][D], the ring matrices (3 (ov)^2), the three-body operator [o][o v^2]; t2 (and l2)
 * are borrowed as for gfcc_build_intermediates.  Build temporaries hold the integral
 * blocks (ov|vv) and the v^4 product.  Blocking.  Errors as gfcc_build_intermediates. */
gfcc_status gfcc_build_ea_intermediates(const gfcc_system* sys, void* stream, gfcc_ctx** out);

/* One open-shell (spin-unrestricted) system in spin blocks.  Device pointers, FP64.
 *   n                   spatial orbitals per spin; n_occ_a alpha and n_occ_b beta electrons
 *                       (1 <= n_occ_b <= n_occ_a < n); va = n - n_occ_a, vb = n - n_occ_b
 *   eps_a, eps_b [n]    orbital energies of each spin (Fock matrices diagonal), occupied first
 *   La, Lb [Q][n][n]    Cholesky vectors of each spin's orbitals, symmetric in (p,q):
 *                       (pq|rs) = sum_Q L_s[Q][p][q] L_s'[Q][r][s] for p,q of spin s and r,s of s'
 *   t1a [oa][va], t1b [ob][vb]
 *   t2aa [oa][oa][va][va], t2bb [ob][ob][vb][vb]   antisymmetric in (i,j) and in (a,b)
 *   t2ab [oa][ob][va][vb]                          t_{i alpha, j beta}^{a alpha, b beta}
 *   l1a ... l2bb        Lambda in the same layouts; all NULL means Lambda = T^dagger.
 * Everything is read during gfcc_build_uhf_intermediates only (the context keeps its own
 * spin-orbital copies). */
typedef struct {
  int64_t n, n_occ_a, n_occ_b, n_chol;
  const double* eps_a;
  const double* eps_b;
  const double* La;
  const double* Lb;
  const double* t1a;
  const double* t1b;
  const double* t2aa;
  const double* t2ab;
  const double* t2bb;
  const double* l1a;
  const double* l1b;
  const double* l2aa;
  const double* l2ab;
  const double* l2bb;
} gfcc_uhf_system;

/* Build the context of the retarded IP term for an open-shell reference (Theory section: the
 * first term of the Green's function and the linear system for X_p; the open-shell
 * GFCCSD-IP of the Evaluation section, Table 2, treats alpha and beta electrons separately).
 * Everything is over spin orbitals: o = n_occ_a + n_occ_b occupied ones ordered
 * [alpha 0..oa-1, beta 0..ob-1], v = va + vb virtual ones ordered [alpha, beta]; orbital
 * indices p, q of the other entry points run over [0, o + v) in that order (occupied first).
 * Both ionised sectors (an alpha or a beta electron removed) live in one space of dimension
 * D = o + o*o*v:
 *     x[0 .. o)                = r_i
 *     x[o + (i*o + j)*v + a]   = r_ij^a,  stored for both orders: r_ji^a = -r_ij^a, r_ii^a = 0
 * with R = sum_i r_i a_i + 1/2 sum_ija r_ij^a a_a^+ a_j a_i.  gfcc_sigma returns Hbar_N X
 * (antisymmetric inputs give antisymmetric outputs; FP64 only); gfcc_solve_batch solves
 * (omega + Hbar_N - i eta) X_p = abar_p|Phi> (occupied p: e_p; virtual p = o + a:
 * r_i = t_i^a, r_ij^b = t_ij^ab) and G[r][k] = G_{q[k] p[r]} = c_q . X_p with the left rows
 * carrying 1/2 on their 2h1p block (each pair counted once); G vanishes between orbitals of
 * different spin.  FP64 only; GFCC_PC_MLP is E_STATE.  gfcc_solve_shifts (FP64 fallback only),
 * gfcc_greens(_noalloc), gfcc_export
 * (FOO, FVV, FOV over spin orbitals, DIAG [D]), gfcc_prof_*, gfcc_destroy work on it; every
 * other entry point returns E_STATE.  Storage: spin-orbital <oo||vv>, W_oooo, W_ooov, W_ovvo,
 * W_ovoo and the amplitudes (o^2 v^2 each); the build's temporaries hold the <ov||vv> blocks
 * and the spin-orbital Cholesky vectors.  Blocking.  E_ARG for bad sizes or missing blocks. */
gfcc_status gfcc_build_uhf_intermediates(const gfcc_uhf_system* sys, void* stream, gfcc_ctx** out);

/* Device-memory plan of one system in bytes (host arithmetic only, no GPU
 * needed): the caller's inputs, each operand the context keeps in FP64 and in
 * the reduced precision `prec`, the build's fixed temporaries and smallest
 * chunk, and the solver's bytes per slot of a window (restart length,
 * flexible = 1 for the learned preconditioner's FGMRES) with the sigma operand
 * copies of `window` slots.  total = the borrowed t2/l2 + context (FP64 +
 * reduced precision) + window slots + sigma workspace, what a solve holds;
 * build_peak = all inputs (L included) + FP64 context + the build's fixed
 * temporaries and smallest chunk. */
typedef struct {
  size_t struct_size;                    /* sizeof(gfcc_memory_plan) */
  double input_L, input_t2, input_l2;    /* caller's buffers (L is read during the build only) */
  double ring, ladder, wovoo, wooov;     /* [Wovvo|Wovov], Woooo, Wovoo, Wooov */
  double cholesky, rows_1h, left;        /* Cholesky operands of the three-body term, 1h rows, c_q rows */
  double vectors, small;                 /* diagonal and other O(D) arrays; one-body blocks */
  double context_fp64, context_lowp;
  double build_fixed, build_chunk_min;
  double per_slot, sigma_workspace, total, build_peak;
} gfcc_memory_plan;
gfcc_status gfcc_plan_memory(int64_t n_occ, int64_t n_vir, int64_t n_chol, gfcc_precision prec, int32_t restart,
                             int32_t flexible, int64_t window, int32_t lambda_given, gfcc_memory_plan* out);

/* Dimensions of the context: D = o + o*o*v, o, v. Host pointers; any may be NULL. */
gfcc_status gfcc_dims(const gfcc_ctx* ctx, int64_t* D, int64_t* n_occ, int64_t* n_vir);

/* Copy one built FP64 block into a caller device buffer (for verification).
 * Layouts (index order = array order):
 *   FOO [m][i]  FVV [a][e]  FOV [m][e]  WOOOO [m][n][i][j]  WOOOV [m][n][i][e]
 *   WOVOO [m][a][i][j]  WOVVO [m][a][e][j]  WOVOV [m][a][j][e]
 *   DIAG [D]    (exact diagonal of Hbar_N)
 *   LEFT [o][D] (row q = c_q)                                             */
typedef enum {
  GFCC_FOO = 0, GFCC_FVV, GFCC_FOV, GFCC_WOOOO, GFCC_WOOOV, GFCC_WOVOO, GFCC_WOVVO, GFCC_WOVOV,
  GFCC_DIAG, GFCC_LEFT, GFCC_N_BLOCKS
} gfcc_block;
gfcc_status gfcc_export(gfcc_ctx* ctx, gfcc_block which, double* dst, void* stream);

/* The sigma product Y[r] = Hbar_N X[r] for r < nrhs: the action of the
 * connected similarity-transformed Hamiltonian on the 1h + 2h1p expansion of
 * X_p (Theory section, the linear system for X_p and the X_p expansion; the
 * per-iteration O(o^3 v^2) work of the GMRES micro loop, GFCC Workflow and
 * Bottlenecks, Algorithm 1).  X, Y: device [nrhs][D] complex interleaved; may
 * not alias.  prec selects the arithmetic of the two-body contractions (FP32 or
 * BF16 on MFMA with FP32 accumulation; the one-body terms stay FP64).  E_ARG for
 * a bad precision or aliased/NULL buffers.  Enqueued on `stream`. */
gfcc_status gfcc_sigma(gfcc_ctx* ctx, int64_t nrhs, const double* X, double* Y,
                       gfcc_precision prec, void* stream);

typedef struct {
  size_t struct_size;       /* sizeof(gfcc_solve_opts) */
  double tol;               /* on ||b - A x|| / ||b||, true FP64 residual */
  int32_t restart;          /* Krylov vectors per cycle (>= 1) */
  int32_t max_iter;         /* total inner iterations per right-hand side */
  int32_t batch;            /* active right-hand sides per launch; 0 = auto: up to 512, within half of free HBM */
  gfcc_precond precond;
  gfcc_precision precision;
  int32_t use_graph;        /* capture one inner iteration in a hipGraph and replay it */
  const char* tune_cache;   /* host path of the tile autotuner JSON cache; NULL = no tuning */
  double ir_inner_rtol;     /* GMRES-IR: inner cycle stops at this fraction of the cycle's starting
                               residual; 0 = default for the precision (ignored for FP64) */
  const char* checkpoint;   /* host path of a resume file, or NULL.  A new or empty file gets a
                               header (magic, version, record size, a fingerprint of the request:
                               each system's dimensions and exact diagonal, the system of each
                               right-hand side, q, eta, tol, precision, precond, restart, max_iter);
                               every finished right-hand side then appends (index, p, omega, eta,
                               G row, info), and a later call with the same request restores the
                               rows it holds instead of solving them.  A file without a valid
                               header, or with another request's fingerprint, is refused with
                               E_ARG and left unchanged; a torn last record is trimmed.
                               gfcc_solve_batch and gfcc_solve_multi; ignored by the solves that
                               model-order reduction and the multi-shift fallback run.  Restored
                               rows get X = 0 when X is requested. */
  int32_t sync_every;       /* inner iterations between host synchronisations of the solver loop
                               (flags, Krylov steps and residual estimates copied back in one
                               transfer).  0 = automatic, from each active right-hand side's
                               predicted iterations to its cycle target (the observed decrease of
                               its residual estimate, capped by the restart length): where the
                               window's sigma is estimated under 2 ms per iteration the run lasts
                               until half of a system's slots are predicted to stop, otherwise it
                               ends at 85% of the first slot's prediction; at most 16.  1 = after
                               every iteration; k > 1 = runs of k.  A slot whose cycle stops inside
                               a run is frozen on the device, so G, X and info do not depend on this
                               value (FP16-IR: up to rounding, as the per-call vector scale sees the
                               frozen planes); it is 1 whenever the learned preconditioner or
                               profiling is on.  Runs never pass a right-hand side's max_iter. */
} gfcc_solve_opts;

/* Per right-hand side result (host memory). status: 0 converged, 1 max_iter,
 * 2 breakdown, 3 non-finite, 4 converged after falling back to Jacobi.
 * true_rel_resid = |b_p - (omega + Hbar_N - i*eta) X| / |b_p| in FP64. */
typedef struct {
  int32_t status, iters, restarts, reserved;
  double true_rel_resid;
} gfcc_rhs_info;

/* Solve (omega_r + Hbar_N - i*eta) X_r = b_{p_r} for r < nrhs and form
 * G[r][k] = c_{q_k}^T X_r.  p, omega: host arrays [nrhs]; q: host [nq] or
 * NULL meaning q = p_r per right-hand side (then nq must be 1: G[r][0] = G_pp).
 * p and q lie in [0, o + v).  A right-hand side with b_p = 0 (a virtual p no
 * amplitude reaches) returns X = 0, G = 0, status 0 and no iterations.
 * G: device [nrhs][nq] complex interleaved.  X: device [nrhs][D] complex or
 * NULL (solutions are not kept).  info: host [nrhs].  eta is signed; the
 * operator is exactly (omega + Hbar_N - i*eta).  Right-hand sides are
 * processed through a persistent window of `batch` slots; a slot whose system
 * converges is refilled from the queue.  Blocking.  Returns GFCC_W_NOCONV if
 * any right-hand side did not converge. */
gfcc_status gfcc_solve_batch(gfcc_ctx* ctx, int64_t nrhs, const int64_t* p, const double* omega,
                             double eta, int64_t nq, const int64_t* q, const gfcc_solve_opts* opts,
                             double* G, double* X, gfcc_rhs_info* info, void* stream);

/* gfcc_greens for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments and results, with every intermediate (the vectors in plane layout,
 * the left rows, the orbital list, split-K partials) in a fixed 64 MiB device
 * array that the library holds on each GPU from load until the process ends.
 * Calls no hipMalloc/hipFree.  E_ARG when the request does not fit the array
 * (at least one vector's two planes plus the nq left rows, each o + o*o*v
 * doubles, must fit), E_STATE when the context's device is not current.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race.  Blocking. */
gfcc_status gfcc_greens_noalloc(gfcc_ctx* ctx, int64_t nrhs, const int64_t* p, const double* X, int64_t nq,
                                const int64_t* q, double* G, void* stream);

/* ---------------------------------------------------------------------------
 * Multi-shift GMRES (the shifted systems solved together over many frequencies,
 * Introduction and Theory sections).  The Krylov space of (omega - i*eta +
 * Hbar_N) and b_p is the same for every omega, so one real Arnoldi basis per
 * orbital p (FP64, no preconditioner, no restart) gives the GMRES iterate of
 * every frequency.  Each (p, omega) ends when its FP64 true residual
 * |b_p - (omega + Hbar_N - i*eta) X| / |b_p| <= tol (formed from the stored
 * sigma products, without another sigma). */
typedef struct {
  size_t struct_size;      /* sizeof(gfcc_shift_opts) */
  double tol;              /* relative residual per (p, omega) */
  int32_t max_dim;         /* Krylov dimension cap per orbital, <= 512; 0 = 160 */
  int32_t batch;           /* orbitals in flight; 0 = as many as fit in 40% of free memory */
  int32_t verify;          /* 1 = accept on the FP64 true residual, 0 = on the Givens estimate */
  int32_t use_fallback;    /* 1 = (p, omega) not converged within max_dim are solved again by
                              gfcc_solve_batch with `fallback` */
  gfcc_solve_opts fallback;
  const char* tune_cache;  /* host path of the tile autotuner JSON cache (FP64 sigma shapes of the
                              orbital window); NULL = no tuning */
} gfcc_shift_opts;

/* For every orbital p[i] (host [np], in [0, o + v)) and every frequency omega[k]
 * (host [n_omega]) solve (omega_k + Hbar_N - i*eta) X = b_p.  G (device):
 * [np][n_omega][nq] complex interleaved, G = c_q^T X for q (host [nq], in
 * [0, o + v)), or q = NULL and nq = 1 for G_pp.  X (device, nullable):
 * [np][n_omega][D] complex.  info (host [np][n_omega]): status as for
 * gfcc_solve_batch (1: not converged within max_dim and no fallback), iters =
 * basis size used (plus fallback iterations), true_rel_resid.  Memory: per
 * orbital in flight (2 max_dim + 1) planes of (o + o*o*v) doubles.  Blocking;
 * returns GFCC_W_NOCONV if any (p, omega) did not converge. */
gfcc_status gfcc_solve_shifts(gfcc_ctx* ctx, int64_t np, const int64_t* p, int64_t n_omega,
                              const double* omega, double eta, int64_t nq, const int64_t* q,
                              const gfcc_shift_opts* opts, double* G, double* X, gfcc_rhs_info* info,
                              void* stream);

/* Spectral function from the diagonal of the retarded G (Theory section, the
 * trace of its imaginary part): A[k] = sgn(eta)/pi * sum_p Im G_pp(omega_k).
 * With the operator (omega + Hbar_N - i*eta) and eta > 0, Im G_pp > 0 at the
 * poles, so this equals the paper's -(1/pi) Im of the +i*eta form; eta < 0
 * conjugates G and the sign keeps A the same.  G: device [np][ld] complex
 * interleaved, element (p, k) = G_pp(omega_k), ld >= n_omega (e.g. the G of
 * gfcc_solve_shifts with q = NULL, or of gfcc_solve_batch ordered p-major).
 * A: device [n_omega].  Needs no context.  Enqueued on `stream`. */
gfcc_status gfcc_spectral(int64_t np, int64_t n_omega, const double* G, int64_t ld, double eta, double* A,
                          void* stream);

/* Right-hand sides of several systems in one persistent solve (uneven
 * convergence across systems, the paper's dynamic pickup of work by idle
 * process groups in Implementation Details, here at slot granularity): right-hand
 * side r belongs to system sys[r] (host [nrhs], index into ctxs[0:nsys], distinct
 * contexts, nsys <= 16).  Each system gets a share of the slot window in
 * proportion to its right-hand sides (opts->batch = total window, 0 = auto);
 * all systems advance together, one inner iteration of every system per step,
 * and the ring GEMMs of up to four systems run as one grouped launch.  p, omega,
 * q, G, info as for gfcc_solve_batch (q must be valid for every system);
 * solutions are not returned.  Blocking. */
gfcc_status gfcc_solve_multi(int32_t nsys, gfcc_ctx* const* ctxs, int64_t nrhs, const int32_t* sys,
                             const int64_t* p, const double* omega, double eta, int64_t nq, const int64_t* q,
                             const gfcc_solve_opts* opts, double* G, gfcc_rhs_info* info, void* stream);

/* Green's function from caller solutions (Theory section: the compact form
 * G_qp = <Phi|(1 + Lambda) abar_q^+ X_p|Phi>, evaluated as the bilinear product
 * c_q^T X_p of the model-order-reduction equations, no conjugation):
 * G[r][k] = c_{q_k}^T X[r] for vectors X [nrhs][D] complex interleaved (device).
 * q: host [nq] in [0, o + v), the same list for every vector; or q = NULL with
 * nq = 1, the diagonal form G[r][0] = c_{p_r}^T X[r] with p host [nrhs] in
 * [0, o + v) (p is read only when q is NULL).  G: device [nrhs][nq] complex
 * interleaved.  E_ARG for out-of-range orbitals or a NULL q without p or with
 * nq != 1.  Blocking. */
gfcc_status gfcc_greens(gfcc_ctx* ctx, int64_t nrhs, const int64_t* p, const double* X, int64_t nq,
                        const int64_t* q, double* G, void* stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner (GFCC_PC_MLP).  An elementwise network corrects the
 * Jacobi step of the classic diagonal preconditioner (GFCC Workflow and
 * Bottlenecks section): per element d of a complex vector r, with
 * z = omega - i eta, exact diagonal D of Hbar_N, sD = mean |D| and
 * n = ||r|| / sqrt(D_dim),
 *   features x_d = [Re rh, Im rh, Re jh, Im jh, D_d/sD - 1, omega, [d < o], 100 eta],
 *     rh = r/n, jh = rh sD/(z + D)
 *   y_d = W3 tanh(W2 tanh(W1 x_d + b1) + b2) + b3        (8 -> W -> W -> 2)
 *   M(r)_d = r_d/(z + D_d) + (y_d0 + i y_d1) n/sD
 * Flat parameter layout (FP64): W1[W][8], b1[W], W2[W][W], b2[W], W3[2][W], b3[2].
 * ------------------------------------------------------------------------- */
typedef struct {
  size_t struct_size;   /* sizeof(gfcc_mlp_opts) */
  int32_t width;        /* hidden width W: 64, 128 or 256 */
  int32_t steps;        /* Adam steps */
  int32_t batch;        /* sampled elements per minibatch */
  int32_t pair_restart; /* restart length of the data-generating FP64 Jacobi solves */
  double lr;            /* Adam learning rate */
  uint64_t seed;        /* initialisation and sampling seed */
  int32_t max_pairs;    /* cap on stored (residual, error) pairs */
  int32_t data_max_iter; /* iteration cap of each data-generating solve (0: 4000) */
  double data_tol;      /* tolerance of the data-generating solves (0: 1e-11); X* must be
                           accurate well below the residuals of the recorded pairs */
  int32_t data_precision; /* gfcc_precision of the data-generating solves (their restart
                             residuals are FP64 true residuals in every precision) */
  int32_t reserved;
  double xstar_ratio;   /* 0: only right-hand sides that reach data_tol give pairs.  > 0: a
                           right-hand side stopped at data_max_iter also gives its pairs whose
                           residual is >= xstar_ratio times its last iterate's, with that iterate
                           as X* (the target's relative error is then about 1/xstar_ratio).
                           Absent when struct_size predates the field. */
} gfcc_mlp_opts;

typedef struct {
  int64_t n_pairs;      /* (residual, error) pairs collected */
  int32_t steps, reserved;
  double loss_first;    /* minibatch loss at step 0 (zero output layer: the plain Jacobi step) */
  double loss_final;    /* mean minibatch loss over the last 5% of steps */
  double data_seconds, train_seconds;
} gfcc_mlp_report;

/* Train the network on pairs the solver generates itself: FP64 Jacobi GMRES
 * solves of the given (p, omega) right-hand sides (tolerance opts->data_tol) with restart
 * length opts->pair_restart record, at every restart, the true residual r_k and the
 * iterate x_k; after convergence e_k = X* - x_k (so A e_k = r_k).  Minibatches
 * of elements are sampled on the GPU; loss = mean |y - t|^2 with
 * t = e sD/n - jh; Adam.  p, omega, report: host.  Blocking. */
gfcc_status gfcc_mlp_train(gfcc_ctx* ctx, int64_t nrhs, const int64_t* p, const double* omega, double eta,
                           const gfcc_mlp_opts* opts, gfcc_mlp_report* report, void* stream);

/* Load / read the flat FP64 parameter vector (device).  get: *width is set;
 * params may be NULL to query the width only. */
gfcc_status gfcc_mlp_set_weights(gfcc_ctx* ctx, int32_t width, const double* params, void* stream);
gfcc_status gfcc_mlp_get_weights(gfcc_ctx* ctx, int32_t* width, double* params, void* stream);

/* One Adam step (Kingma & Ba: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias
 * corrections 1 - beta^t) on the network weights with the caller's flat
 * gradient grad [n_params] (device), the step the training loop takes after
 * each minibatch gradient.  The moments and the step count t live in the
 * context and start at zero when weights are set or training starts.
 * E_STATE without a network.  Blocking. */
gfcc_status gfcc_mlp_adam_step(gfcc_ctx* ctx, const double* grad, double lr, void* stream);

/* FP64 network on caller features: Y[n][2] from X[n][8] (device). */
gfcc_status gfcc_mlp_forward(gfcc_ctx* ctx, int64_t n, const double* X, double* Y, void* stream);

/* Minibatch loss and flat gradient of the FP64 network: loss device [1],
 * grad device [n_params]. */
gfcc_status gfcc_mlp_loss_grad(gfcc_ctx* ctx, int64_t n, const double* X, const double* T, double* loss,
                               double* grad, void* stream);

/* Features of complex vectors R [nvec][D] (device, interleaved) at the
 * per-vector frequencies omega (host [nvec]): X [nvec*D][8] (device). */
gfcc_status gfcc_mlp_features(gfcc_ctx* ctx, int64_t nvec, const double* R, const double* omega, double eta,
                              double* X, void* stream);

/* The preconditioner itself (fused BF16-MFMA inference kernel):
 * U[v] = M(R[v]) for complex vectors R, U [nvec][D] (device, interleaved). */
gfcc_status gfcc_mlp_apply(gfcc_ctx* ctx, int64_t nvec, const double* R, const double* omega, double eta,
                           double* U, void* stream);

/* ---------------------------------------------------------------------------
 * Model-order reduction over frequency levels (Theory section, eq. model;
 * GFCC Workflow and Bottlenecks: the level loop of Algorithm 1, eq. Lmax).
 * The context keeps an orthonormal REAL basis S (m columns): the real and
 * imaginary parts of solved X_p(omega) are separate candidates, so the
 * projected operator Hhat = S^T Hbar_N S is real.  The model system
 * (omega - i eta + Hhat) Xhat = S^T b_p gives G_qp(omega) ~ (S^T c_q)^T Xhat.
 * ------------------------------------------------------------------------- */
typedef struct {
  size_t struct_size;     /* sizeof(gfcc_mor_opts) */
  double tol;             /* an interval is converged when the model built before its level predicts
                             G_pp at its midpoint within tol (relative, every p) */
  double drop_tol;        /* Gram-Schmidt drops a candidate whose norm falls below drop_tol times its
                             norm before orthogonalisation */
  int32_t max_levels;     /* 0: the bound floor(log2((omega_max - omega_min) / d_omega)) */
  int32_t reserved;
  gfcc_solve_opts solve;  /* options of the direct solves of each level */
} gfcc_mor_opts;

typedef struct {
  int32_t levels;         /* levels run */
  int32_t m;              /* final basis size */
  int32_t n_solved;       /* grid frequencies solved directly */
  int32_t converged;      /* 1: every interval closed before the level bound */
  int32_t per_level[16];  /* frequencies solved at level 1, 2, ... */
  double max_mid_err;     /* largest midpoint error of the last tested level */
  double t_solve, t_basis, t_project, t_model;  /* seconds in each phase */
} gfcc_mor_report;

/* Forget the basis. */
gfcc_status gfcc_mor_reset(gfcc_ctx* ctx);

/* Gram-Schmidt the real and imaginary parts of n complex vectors X [n][D]
 * (device, interleaved; not modified) into the basis (classical, one
 * reorthogonalisation, dependent candidates dropped at drop_tol), apply the
 * FP64 sigma to the new columns and extend Hhat.  *m_out (host, nullable):
 * basis size afterwards.  Blocking. */
gfcc_status gfcc_mor_extend(gfcc_ctx* ctx, int64_t n, const double* X, double drop_tol, int64_t* m_out,
                            void* stream);

/* Model Green's function at n_omega frequencies (host) for occupied p (host
 * [np]; the model right-hand side is S^T e_p) and q (host [nq], occupied or
 * virtual); q == NULL: the diagonal q = p, G [n_omega][np],
 * else G [n_omega][np][nq]; complex interleaved, device.  E_STATE when the
 * basis is empty or a model system is singular.  Blocking. */
gfcc_status gfcc_mor_model(gfcc_ctx* ctx, int64_t np, const int64_t* p, int64_t nq, const int64_t* q,
                           int64_t n_omega, const double* omega, double eta, double* G, void* stream);

/* Copy the basis out: which = 0: Hhat [m][m] row-major, Hhat[i][j] = s_i . Hbar_N s_j;
 * which = 1: S [m][D] (real vectors in the boundary layout).  dst: device,
 * may be NULL to query *m_out (host). */
gfcc_status gfcc_mor_export(gfcc_ctx* ctx, int32_t which, double* dst, int64_t* m_out, void* stream);

/* The level loop on a uniform ascending grid omega[0:n_omega] (host): level 1
 * solves both ends and the middle, level L > 1 solves the midpoints of the
 * open intervals; an interval closes when its midpoint passes opts->tol and
 * intervals without interior grid points close.  Each level's solutions
 * extend the basis.  G [n_omega][np] (device, complex interleaved) is the
 * final model G_pp on the whole grid; level_of (host [n_omega], nullable):
 * the level at which a frequency was solved directly, 0 if never; report:
 * host, nullable.  Returns GFCC_W_NOCONV when a direct solve did not converge.
 * Blocking. */
gfcc_status gfcc_mor_greens(gfcc_ctx* ctx, int64_t np, const int64_t* p, int64_t n_omega, const double* omega,
                            double eta, const gfcc_mor_opts* opts, double* G, int32_t* level_of,
                            gfcc_mor_report* report, void* stream);

/* Kernel timing of the library's launches with HIP events on the launch
 * stream.  enable != 0 starts recording (clears totals); enable = 0 stops it and
 * also clears them.  For a kernel class name ("ring_gemm_fp64", "ring_gemm_fp32",
 * "ring_gemm_bf16", "ring_gemm_fp16" -- the two ring GEMMs of sigma --, the same
 * split by GEMM tile as "ring_gemm_<prec>:<tile>" (tiles: 128x128 64x64 128x64
 * 64x128 db128x128 db256x128 db128x256 db256x256 db32_256x256 db32_256x128
 * db32_128x128 db32_256x256w16 db256x256w16 dma3_256x256 dma4_256x256 dma3_256x256w8
 * dma3_256x256w8t dma2k64_256x256; the environment variable GFCC_TILE_<FP64|FP32|BF16|FP16>
 * set to one of these names forces that tile for every product of that precision that would
 * take a tuned or default large tile), "sigma", "arnoldi" (bytes:
 * algorithmic HBM bytes of the Arnoldi step), "mlp", "ea_sigma", "ea_ring",
 * "ea_ladder", "uhf_sigma") gfcc_prof_get returns the number of launches, total
 * milliseconds and algorithmic flops and bytes summed over them (host outputs).
 * Counted whether or not recording is on (count only): "graph_capture" and
 * "graph_replay", the inner iterations the solver captured as a hipGraph and
 * replayed from one (graph replay is off while recording).  Blocking. */
gfcc_status gfcc_prof_enable(gfcc_ctx* ctx, int enable);
gfcc_status gfcc_prof_get(gfcc_ctx* ctx, const char* name, int64_t* count, double* ms,
                          double* flops, double* bytes);

gfcc_status gfcc_destroy(gfcc_ctx* ctx);
const char* gfcc_strerror(gfcc_status st);
const char* gfcc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GFCC_H */
