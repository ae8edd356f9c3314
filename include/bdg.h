/*
 * bdg.h - C ABI of the MI355X (gfx950) spin-1 Bogoliubov-de Gennes excitation library.
 *
 * The library computes the lowest positive excitation frequencies omega of a spin-1
 * Bose-Einstein condensate around its mean-field ground state (Li, Li, Xie, Zhang,
 * "An efficient Fourier spectral algorithm for the Bogoliubov-de Gennes excitation
 * eigenvalue problem", arXiv 2506.08308).  Every step runs in the library's own HIP
 * kernels on the device; there is no host fallback.
 *
 * Problem statement (Section 1, eqs. GPE, groundDef; Section 2.1, eqs. BdG_uv, def_A..def_D):
 *   box D = [-L_x, L_x) x [-L_y, L_y) x [-L_z, L_z) (first `dim` axes), periodic,
 *   N_a points per axis, x_j = -L_a + j h_a, h_a = 2 L_a / N_a (Section 3.1);
 *   external potential V(x) (real), interaction strengths beta_n, beta_s,
 *   mass N = ||Phi||^2 and magnetization ||phi_1||^2 - ||phi_-1||^2 = M * N.
 *
 * Memory layout (all device pointers, caller-owned unless stated otherwise):
 *   grid field: N_x*N_y*N_z values, x fastest (index x + N_x*(y + N_y*z));
 *   real ground state Phi: 3 grid fields (phi_1, phi_0, phi_-1), float64;
 *   trial vector: 6 complex grid fields, interleaved (re, im):
 *     (f_1, f_0, f_-1, g_1, g_0, g_-1) in the (f, g) form of eq. (lrep-d), or
 *     (u_1, u_0, u_-1, v_1, v_0, v_-1) in the (u, v) form of eq. (BdG-d);
 *   block of b vectors: b consecutive trial vectors (vector j at offset j * 6 * npts).
 *   complex128 (double2) in BDG_FP64 mode; bdg_apply takes complex64 (float2) blocks
 *   when the context was created with BDG_FP32_APPLY.
 *
 * Inner product (Section 2.1, discretized as in Section 3.4): <a, b> = h_x h_y h_z sum_j a_j conj(b_j).
 *
 * Errors: every call returns a bdg_status; nothing else crosses the ABI (no exceptions,
 * no aborts).  The message of the last failure is kept in the context and returned by
 * bdg_last_error.  Calls on one context are not thread safe.
 *
 * Streams: the context works on the HIP stream given at creation (NULL = the default
 * stream).  bdg_apply is asynchronous on that stream; every other call returns with
 * its outputs complete.
 */
#ifndef BDG_H
#define BDG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdg_ctx bdg_ctx;

typedef enum {
    BDG_OK = 0,
    BDG_EINVAL = 1,       /* invalid argument: nothing was computed */
    BDG_ENOMEM = 2,       /* device allocation failed */
    BDG_ENOCONV = 3,      /* iteration limit reached; outputs hold the last iterate */
    BDG_EBREAKDOWN = 4,   /* bi-orthogonal basis lost rank below the requested count */
    BDG_EDEVICE = 5,      /* no usable gfx950 device or a HIP runtime error */
    BDG_ESTATE = 6        /* call order: e.g. apply before a ground state was set */
} bdg_status;

typedef enum { BDG_FP64 = 0, BDG_FP32_APPLY = 1 } bdg_precision;
typedef enum { BDG_FORM_UV = 0, BDG_FORM_FG = 1 } bdg_form;

typedef struct {
    int dim;              /* 1, 2 or 3 */
    int n[3];             /* points per axis (x, y, z); powers of two, 8 <= n <= 1024; unused axes ignored */
    double L[3];          /* half box lengths (> 0) */
    double beta_n;        /* density interaction (eq. GPE) */
    double beta_s;        /* spin-exchange interaction: < 0 ferromagnetic, > 0 antiferromagnetic */
    double mass;          /* ||Phi||^2 > 0 (the paper fixes 1) */
    double magnetization; /* M in (-1, 1): ||phi_1||^2 - ||phi_-1||^2 = M * mass */
    int precision;        /* bdg_precision */
} bdg_problem;

/* Create a context: validates the problem (BDG_EINVAL on dim outside 1..3, n not a power of
 * two in [8, 1024], L <= 0, mass <= 0, M outside (-1, 1), non-finite beta or V), copies V
 * (npts float64, device) and builds twiddle and wavenumber tables.  Ownership of the
 * context passes to the caller; release it with bdg_destroy. */
bdg_status bdg_create(const bdg_problem* problem, const double* V_dev, void* hip_stream,
                      bdg_ctx** out);
void bdg_destroy(bdg_ctx* ctx);
const char* bdg_last_error(const bdg_ctx* ctx);

/* Ground state (Section 1, eqs. groundDef, NLEP): normalized gradient flow
 *   Phi <- Normalize(Phi - tau (|k|^2/2 + alpha)^-1 r),  r = H(Phi) Phi - mu Phi - lambda S_z Phi,
 * with (mu, lambda) the least-squares multipliers and the three-factor normalization of the
 * normalized-gradient-flow literature (mass, magnetization, sigma_1 sigma_-1 = sigma_0^2).
 * phi0_dev: 3 npts float64 start (NULL = Gaussian times the spin weights:
 *   beta_s < 0: ((1+M)/2, sqrt((1-M^2)/2), (1-M)/2); beta_s >= 0: (sqrt((1+M)/2), 0, sqrt((1-M)/2))).
 * Stops when ||r|| <= tol * sqrt(mass) (BDG_ENOCONV after max_iter steps).
 * phi_dev (3 npts, caller-owned) receives Phi; mu[3] = (mu_1, mu_0, mu_-1) = (mu+lambda, mu,
 * mu-lambda); the result also becomes the context's ground state. */
bdg_status bdg_ground_state(bdg_ctx* ctx, const double* phi0_dev, double tol, int max_iter,
                            double* phi_dev, double mu[3], double* residual, int* iters);

/* Install a ground state computed elsewhere (3 npts float64, device) with its chemical
 * potentials; builds the pointwise coefficient fields of H_+ = A + B and H_- = A - B. */
bdg_status bdg_set_ground_state(bdg_ctx* ctx, const double* phi_dev, const double mu[3]);

/* Install a complex ground state (the general BdG form of Section 2.1: A complex Hermitian,
 * B complex symmetric, H = [[A, B], [-conj B, -conj A]]; e.g. vortex or moving states).
 * phi_dev: 3 npts complex128 (device, copied; components 1, 0, -1); mu[3] (host): the
 * chemical potentials (the caller's state must be stationary with them, as for
 * bdg_set_ground_state).  Needs a BDG_FP64 context (BDG_EINVAL otherwise).  Afterwards
 * bdg_apply takes the (u, v) form without transpose, bdg_eigs solves H x = w x through the
 * Hermitian pencil sigma_3 x = (1/w) K x, K = sigma_3 H, and bdg_perturbed_density uses the
 * complex Phi; bdg_eigs_grad returns BDG_EINVAL.  bdg_ground_state or bdg_set_ground_state
 * return the context to a real ground state. */
bdg_status bdg_set_ground_state_complex(bdg_ctx* ctx, const void* phi_dev, const double mu[3]);

/* Block application of the BdG operator (Section 3.1, eqs. BdG-d / lrep-d; matrix-free
 * product of Section 3.2: forward FFT, kinetic multiplier |k|^2/2, inverse FFT, pointwise
 * 3x3 coupling in physical space).
 *   form = BDG_FORM_FG: Y = [[0, H_-], [H_+, 0]] X, i.e. (H_- g, H_+ f);
 *   form = BDG_FORM_UV: Y = [[A, B], [-B, -A]] X.
 *   transpose = 1 applies the adjoint: (H_+ g, H_- f), resp. [[A, -B], [B, -A]] X.
 * X_dev, Y_dev: nvec trial vectors (complex128, or complex64 in BDG_FP32_APPLY contexts);
 * they must not overlap.  Asynchronous on the context stream. */
bdg_status bdg_apply(bdg_ctx* ctx, int form, int transpose, int nvec, const void* X_dev,
                     void* Y_dev);

/* Block bi-orthogonal Gram-Schmidt (Section 3.2, bi-orthogonality theorem of Section 2.2):
 * F_dev, G_dev: nvec columns of 3 npts complex128 each (column j at offset j * 3 * npts),
 * replaced in place by F C_f, G C_g with (G C_g)^H (F C_f) h^d = I.  The pairing matrix
 * B = h^d G^H F = U diag(sigma) V^H gives C_f = V sigma^-1/2, C_g = U sigma^-1/2; columns
 * with sigma_i <= 1e-12 sigma_1 are dropped and returned as zeros.  sigma (host, nvec)
 * receives the singular values in descending order, rank the number kept. */
bdg_status bdg_biortho(bdg_ctx* ctx, int nvec, void* F_dev, void* G_dev, double* sigma,
                       int* rank);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bdg_biortho with separate outputs that
 * allocates nothing.  F_out = F C_f and G_out = G C_g exactly as bdg_biortho computes them
 * in place (same factors, same rank rule; the Gram matrix's split-K partial sums are fewer,
 * so results agree to rounding, not bit for bit).  F_dev, G_dev (inputs) and F_out_dev,
 * G_out_dev (outputs): nvec columns of 3 npts complex128 each, caller-owned, no output may
 * overlap another buffer.  Every workspace byte lives in one static device array of
 * BDG_NOALLOC_SCRATCH_BYTES per device (held until the process ends): 1 <= nvec <=
 * BDG_NOALLOC_MAX_VEC, BDG_EINVAL otherwise or on overlapping buffers.  Calls that overlap
 * in time on one device share that array and race; the array keeps the last call's
 * contents.  Synchronous on the context stream. */
#define BDG_NOALLOC_MAX_VEC 64
#define BDG_NOALLOC_SCRATCH_BYTES (48ull << 20)
bdg_status bdg_biortho_noalloc(bdg_ctx* ctx, int nvec, const void* F_dev, const void* G_dev, void* F_out_dev,
                               void* G_out_dev, double* sigma, int* rank);

/* k smallest strictly positive excitation frequencies (Section 3.2): block subspace
 * iteration on [[0, H_-], [H_+, 0]] with deflation of the generalized nullspace
 * (Section 2.3), bi-orthogonal Gram-Schmidt and Rayleigh-Ritz projection.  Corrections
 * use the kinetic-potential preconditioner D (|k|^2/2 + sigma)^-1 D with
 * sigma = max(mu_0 / 2, 1/2) and D^2 = sigma / (sigma + max(V - mu_0, 0)) (mu_0: the
 * middle chemical potential); columns whose residual already meets its target get no
 * correction (soft locking).  Converged when every wanted column has
 *   res_j = ||(H_- g_j - w_j f_j, H_+ f_j - w_j g_j)|| / (|w_j| ||(f_j, g_j)||)
 *         <= max(tol, 100 eps ||H|| / |w_j|),
 * checked with a float64 apply at the end; the second term is the float64 rounding floor of
 * this relative residual (eps = DBL_EPSILON, ||H|| bounded by the largest kinetic symbol plus
 * the largest pointwise row sum of H_+-), so `residual` may exceed a tol below that floor.
 * For a real ground state the operator is real and the iteration runs on real trial vectors
 * (two to a complex column inside the library; the block is rounded up to an even count):
 * X0_dev: block x 6 npts complex128 start block in (f, g) form whose vector j contributes the
 * real start vector Re + Im (NULL = real normal vectors drawn from `seed`); the eigenvectors
 * come back real (zero imaginary parts).  omega (host, k): ascending; UV_dev (device, k x 6 npts
 * complex128): eigenvectors in (u, v) form with int |u|^2 - |v|^2 = 1 (i.e. <f, g> = 1/4);
 * may be NULL.  residual (host, k), iters (host) may be NULL.  Needs
 * 1 <= k <= block <= min(160, 3 npts - 4) (each half of a trial vector lives in 3 npts
 * dimensions, less up to 4 deflated directions); BDG_EINVAL otherwise.  BDG_ENOCONV after
 * max_iter iterations (outputs hold the last iterate); BDG_EBREAKDOWN when the projected
 * problem keeps losing rank or definiteness after the basis refreshes. */
bdg_status bdg_eigs(bdg_ctx* ctx, int k, int block, double tol, int max_iter,
                    const void* X0_dev, unsigned long long seed, double* omega, void* UV_dev,
                    double* residual, int* iters);

/* Gradients of eigenvalues (Hellmann-Feynman form with the ground-state sensitivity):
 * for each of the k eigenpairs (omega, (u, v)) given (u, v normalized as bdg_eigs
 * returns them), dV_dev (device, k x npts float64) receives d omega_j / d V(x_i) / h^d
 * (the functional derivative), dbeta_n[k] and dbeta_s[k] (host) the derivatives with
 * respect to beta_n and beta_s.  The ground state must have been computed by
 * bdg_ground_state or installed with bdg_set_ground_state.  Eigenvalues within
 * 1e-8 omega of each other form a cluster and receive the cluster-mean gradient (the
 * derivative of the cluster's mean frequency).  A cluster that continues past index k
 * is cut: its members' gradients then depend on the basis inside the eigenspace, so
 * choose k at a gap of the spectrum. */
bdg_status bdg_eigs_grad(bdg_ctx* ctx, int k, const double* omega, const void* UV_dev,
                         double* dV_dev, double* dbeta_n, double* dbeta_s);

/* Perturbed densities of normal modes (Section 4.2, Applications; the perturbed-density
 * formula used to visualize an excitation): for nmodes eigenpairs and nt times,
 *   n_j^l(x, t_s) = |phi_j(x) + eps (u_j^l(x) e^{-i omega_l t_s} + conj(v_j^l(x)) e^{i omega_l t_s})|^2,
 * j = 1, 0, -1, with Phi the context's ground state.  omega (host, nmodes) and t (host, nt);
 * UV_dev (device, nmodes x 6 npts complex128): the (u, v) vectors as bdg_eigs returns them;
 * out_dev (device, nmodes x nt x 3 npts float64, mode-major, then time, then component).
 * The caller owns every buffer.  nmodes = 0 or nt = 0 is a no-op; BDG_EINVAL on negative
 * counts, null pointers or non-finite omega, t, eps; BDG_ESTATE without a ground state.
 * Synchronizes the context stream before returning. */
bdg_status bdg_perturbed_density(bdg_ctx* ctx, int nmodes, const double* omega, const void* UV_dev,
                                 double eps, int nt, const double* t, void* out_dev);

/* Bogoliubov-amplitude summaries of normal modes (Section 4.2, Applications: the 3-D example
 * shows isosurfaces of the amplitudes u_j^l, v_j^l and remarks on their symmetry under
 * reflections of the trap and their compression along its stiffer axis; these are the numbers
 * behind such remarks).  For nmodes vectors in (u, v) form (UV_dev, device, nmodes x 6 npts
 * complex128, as bdg_eigs returns them) and each of their six fields w = u_1, u_0, u_-1, v_1,
 * v_0, v_-1, out (host, nmodes x 6 x 8 doubles, mode-major, then field) receives
 *   [0] h^d sum |w|^2,  [1] max |w|,
 *   [2 + a] h^d sum x_a^2 |w|^2 / [0]                  (a = x, y, z; 0 beyond dim),
 *   [5 + a] Re h^d sum w(x) conj(w(R_a x)) / [0]        (0 beyond dim),
 * with x_a = -L_a + m h_a on the grid and R_a the reflection x_a -> -x_a (grid index
 * m -> (N_a - m) mod N_a): +1 for a field even under R_a, -1 for an odd one.  Entries 2..7 are
 * 0 for a zero field.  nmodes = 0 is a no-op; BDG_EINVAL on a negative count, null pointers or
 * nmodes > 10922.  Needs no ground state.  Synchronous; deterministic (fixed reduction order). */
bdg_status bdg_mode_amplitudes(bdg_ctx* ctx, int nmodes, const void* UV_dev, double* out);

/* Per-phase timers and counters of the last bdg_eigs call (milliseconds from HIP events):
 * out[0] total, out[1] apply, out[2] preconditioner, out[3] Gram matrices, out[4] small
 * dense solves, out[5] basis updates, out[6] setup (deflation), out[7] iterations,
 * out[8] float64 block-vector applies, out[9] float32 block-vector applies.
 * n_out: capacity of out (up to 10 values are written). */
bdg_status bdg_stats(const bdg_ctx* ctx, double* out, int n_out);

#ifdef __cplusplus
}
#endif
#endif /* BDG_H */
