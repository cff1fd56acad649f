/*
 * lrigw — imaginary-frequency G0W0 screening and self-energy with localized
 * resolution of the identity (LRI) in a numerical-atomic-orbital basis, on
 * AMD MI355X (gfx950).
 *
 * Method: Ren, Merz, Jiang, Yao, Rampp, Lederer, Blum, Scheffler,
 * "All-electron periodic G0W0 implementation with numerical atomic orbital
 * basis functions: algorithm and benchmarks", arXiv:2011.01400.  Section and
 * equation labels below refer to that paper.
 *
 * Conventions for every entry point
 *  - All array pointers are DEVICE pointers owned by the caller unless marked
 *    "host".  The library never frees caller memory.  Arrays are row-major;
 *    complex numbers are interleaved (re, im) as in std::complex / torch.
 *  - "complex T" means complex128 (two doubles) when the context precision is
 *    LRIGW_FP64 and complex64 (two floats) for the other precision forms.  Eigenvalues, eigenvectors, Coulomb matrices, grids,
 *    Sigma^c and QP energies are always FP64.
 *  - Calls are asynchronous on the stream given to lrigw_create; outputs are
 *    valid after that stream is synchronised.  Host "info" outputs are written
 *    before the call returns (the call synchronises the stream for them).
 *  - Energies are in Hartree.  Spin-restricted closed shell (spin factor 2).
 *  - Return value: LRIGW_OK (0), a negative error code, or a positive warning.
 *    Argument checks happen before any work is queued; no C++ exception
 *    crosses this interface.
 *
 * Index conventions
 *  - k grid: Gamma-centred n1 x n2 x n3 grid, point (i1,i2,i3) has fractional
 *    coordinates i_d/n_d and index (i1*n2 + i2)*n3 + i3; the q grid is the k
 *    grid; weights 1/N_k (Sec. II A).
 *  - Orbital basis functions are grouped by atom (basis_off), auxiliary
 *    functions likewise (aux_off).
 */
#ifndef LRIGW_H
#define LRIGW_H

#ifdef __cplusplus
extern "C" {
#endif

#define LRIGW_OK 0
#define LRIGW_ERR_ARG (-1)         /* bad argument (sizes, NULL, ordering) */
#define LRIGW_ERR_OOM (-2)         /* device allocation failed */
#define LRIGW_ERR_HIP (-3)         /* HIP runtime error */
#define LRIGW_ERR_NOT_HPD (-4)     /* a matrix that must be Hermitian positive definite is not */
#define LRIGW_ERR_NOCONV (-5)      /* an iteration did not converge */
#define LRIGW_WARN_QP_NOCONV 1     /* some QP equations had no root (E = e + e_static returned) */
#define LRIGW_WARN_PADE_TRUNC 2    /* some Pade fits were truncated at a zero coefficient */
#define LRIGW_WARN_CD_RANGE 3      /* some contour-deformation residues lie beyond the real grid (NaN there) */

enum lrigw_precision {
  LRIGW_FP64 = 0,        /* every contraction in FP64 (the plain path) */
  LRIGW_FP32 = 1,        /* M, chi0 and Sigma^c contractions in FP32 on MFMA, FP32 accumulate */
  LRIGW_SPLIT_BF16 = 2,  /* chi0 and Sigma^c as hi/lo BF16 products on MFMA (hi*hi + hi*lo + lo*hi), FP32 accumulate */
  LRIGW_SPLIT3_BF16 = 3, /* chi0 and Sigma^c with a three-part BF16 split (six products, FP32-like accuracy) */
  LRIGW_SPLIT_MIXED = 4, /* chi0 with the two-part split, Sigma^c with the three-part split */
  LRIGW_SPLIT_F16 = 5    /* chi0 and Sigma^c as two-part FP16 splits of power-of-two scaled operands (three
                            products, 22 significand bits), FP32 accumulate */
};

typedef struct {
  int n_atoms;
  const int *basis_off;  /* host [n_atoms+1]: orbital basis functions of atom A are basis_off[A]..basis_off[A+1]-1 */
  const int *aux_off;    /* host [n_atoms+1]: auxiliary functions of atom A likewise */
  int nk[3];             /* Gamma-centred grid; q grid == k grid */
  int n_bands;           /* bands kept (columns of the eigenvector matrices) */
  int n_occ;             /* occupied bands (T = 0, insulator) */
  int n_freq;            /* imaginary frequencies of the modified Gauss-Legendre grid */
  double x0;             /* grid scale: omega = x0 (1+t)/(1-t) (Ha) */
  double mu;             /* chemical potential, inside the gap (Ha) */
  int qp_lo, n_qp;       /* bands qp_lo..qp_lo+n_qp-1 get Sigma^c and QP energies */
} lrigw_system;

typedef struct lrigw_ctx lrigw_ctx;

/* Create a context for one cell.  `sys` is copied.  `hip_stream` is a
 * hipStream_t (NULL = default stream).  Allocates the per-q workspaces.
 * Errors: ERR_ARG (inconsistent sizes: n_occ < 1, n_occ >= n_bands, qp range
 * outside the bands, offsets not increasing), ERR_OOM, ERR_HIP. */
int lrigw_create(lrigw_ctx **out, const lrigw_system *sys, int precision, void *hip_stream);
int lrigw_destroy(lrigw_ctx *ctx);
const char *lrigw_strerror(int code);

/* Sizes (in elements) of the caller buffers of the calls below. */
typedef struct {
  long long n_k, n_b, n_aux, n_bands, n_freq, nb_max;
  long long h_elems;      /* lrigw_lri_ft output: N_k * nb_max * n_bands * N_aux complex T */
  long long m_chi_elems;  /* lrigw_build_M slice 0: N_k * n_occ * (n_bands-n_occ) * N_aux complex T */
  long long m_sig_elems;  /* lrigw_build_M slice 1: N_k * n_qp * n_bands * N_aux complex T */
  long long w_elems;      /* chi0 / W^c of one q: n_freq * N_aux * N_aux complex T */
  long long sigma_elems;  /* Sigma^c: N_k * n_qp * n_freq complex128 */
  long long m_x_elems;    /* lrigw_build_M slice 2: N_k * n_qp * n_occ * N_aux complex T */
} lrigw_sizes;
int lrigw_get_sizes(const lrigw_ctx *ctx, lrigw_sizes *out /* host */);

/* Grids (Sec. II A; modified Gauss-Legendre frequencies): omega[n_freq] and
 * weight[n_freq] (FP64, ascending omega) from Gauss-Legendre nodes computed on
 * the device; kpq[N_k*N_k] and kmq[N_k*N_k] (int32): index of k+q and k-q.
 * Any output pointer may be NULL.  The context keeps its own copies. */
int lrigw_grids(lrigw_ctx *ctx, double *omega, double *weight, int *kpq, int *kmq);

/* LRI Bloch transform and half-transform (Sec. II C, Eqs. expan_coeff_FT1/2).
 *   lri_R: FP64, concatenation over atoms A of [nR][naux_A][nb_A][N_b]:
 *          C~^{mu(0)}_{a(0), b(R)} with mu and a on atom A (the real-space
 *          two-centre coefficients; real because the basis functions are).
 *   R_list: host int [nR][3], lattice coordinates of R.
 *   evec: complex128 [N_k][N_b][n_bands], KS eigenvectors c_{i n}(k).
 *   H_out: complex T [N_k][nb_max][n_bands][N_aux]:
 *          H[k][a][n][mu] = sum_j C~^{mu(0)}_{a(0), j(k)} c_{j n}(k), a the
 *          a-th function of atom(mu) (rows a >= nb_A of that atom are zero).
 * Errors: ERR_ARG (nR < 1, NULL), ERR_OOM (temporary for the transform). */
int lrigw_lri_ft(lrigw_ctx *ctx, const double *lri_R, const int *R_list, int nR, const void *evec, void *H_out);

/* Two-centre LRI coefficients, Eq. two_center_coeff_determination: the
 * expansion of the orbital products of an atom pair (I in the home cell, J in
 * cell R) that minimises the Coulomb self-repulsion of its error,
 *   C~^{mu(0)}_{i(0),j(R)} = sum_{nu in {I, J(R)}} (i(0),j(R)|nu) (V^{IJ})^{-1}_{nu mu},  mu on I,
 * for `batch` pairs of one shape at once (the step that produces lri_R):
 *   V: FP64 [batch][n][n], the Coulomb matrix of the pair's n auxiliary
 *      functions, I's n_keep first (for I = J, R = 0 only I's); symmetric
 *      positive definite;
 *   T: FP64 [batch][n][nrhs], (ij|nu), one column per product (i, j);
 *   C: FP64 [batch][n_keep][nrhs] output, scale * (rows 0..n_keep-1 of
 *      V^{-1} T), i.e. C~^{mu}_{i(0),j(R)} in the [mu][(i, j)] order of an
 *      lri_R block; scale = 1, or 1/2 for an on-site pair (the two sectors of
 *      Eq. AO_triple_split2 then share the coefficient).
 * All device pointers, caller-owned; workspace of batch*(n*n + n*nrhs)
 * complex128 is allocated and freed inside the call, which synchronises the
 * context stream.  info (host, may be NULL): -1, or the first pair whose V was
 * not positive definite (then ERR_NOT_HPD).
 * Errors: ERR_ARG (batch outside 1..65535, n < 1, n_keep outside 1..n,
 * nrhs < 1, NULL), ERR_OOM, ERR_NOT_HPD. */
int lrigw_lri_fit(lrigw_ctx *ctx, int batch, int n, int n_keep, int nrhs, const double *V, const double *T, double scale,
                  double *C, int *info);

/* lrigw_lri_fit without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments, kernels and results, with the
 * workspace taken from a fixed array of LRIGW_FIT_SCRATCH_BYTES in the
 * library's device memory instead of hipMalloc.  Each device holds its own
 * array until the process ends (its address is looked up at lrigw_create).
 * Calls on one device share that array: calls that overlap on one device (two
 * streams, two threads) race and must be serialised by the caller.  Nothing
 * carries over between calls.  The call synchronises the context stream for
 * `info`, like lrigw_lri_fit.
 * Size limit: 256 + batch*n*n*16 + batch*n*nrhs*16 + batch*ceil(n/64)*64*64*16
 * bytes (each term rounded up to 256) must not exceed LRIGW_FIT_SCRATCH_BYTES.
 * Errors: as lrigw_lri_fit; ERR_ARG also when the shape exceeds the limit. */
#define LRIGW_FIT_SCRATCH_BYTES (64ull << 20)
int lrigw_lri_fit_noalloc(lrigw_ctx *ctx, int batch, int n, int n_keep, int nrhs, const double *V, const double *T,
                          double scale, double *C, int *info);

/* MO triple coefficients (Eqs. AO_triple_split2 and AO_MO_transform) with the
 * Bloch pair (k, k2), mu on P^{(k-k2)*}:
 *   C^mu_{rc}(k,k2) = sum_{a on atom(mu)} conj(c_{a r}(k)) H[k2][a][c][mu]
 *                                      + conj(H[k][a][r][mu]) c_{a c}(k2)
 * (the second sector uses C~(-k) = conj C~(k), true for real coefficients).
 *   slice 0 (response):    k2 = k+q, r over occupied, c over unoccupied bands:
 *       M_out complex T [N_k][n_occ][n_bands-n_occ][N_aux]  (B^mu_ia(k,q))
 *   slice 1 (self-energy): k2 = k-q, r over the QP bands, c over all bands:
 *       M_out complex T [N_k][n_qp][n_bands][N_aux]  (C^mu_{nm}(k,k-q))
 *   slice 2 (exchange):    k2 = k-q, r over the QP bands, c over the occupied bands:
 *       M_out complex T [N_k][n_qp][n_occ][N_aux]
 * Errors: ERR_ARG (iq out of range, slice not 0, 1 or 2, NULL). */
int lrigw_build_M(lrigw_ctx *ctx, int iq, int slice, const void *H, const void *evec, void *M_out);

/* Independent-particle response, Eq. chi0_matrix (occupation difference
 * restored, paired with V(q) as the Dyson equation requires; time-reversal
 * symmetric inputs):
 *   chi_out[w][mu][nu] = -(2/N_k) sum_{k,i,a} 2D/(D^2 + w^2) B^mu_ia conj(B^nu_ia),
 *   D = e_a(k+q) - e_i(k),   for every grid frequency w.
 * M: slice-0 output of lrigw_build_M for this iq.  eig: FP64 [N_k][n_bands].
 * apply_gamma (iq == 0 only, after lrigw_gamma_prepare): replace, in every
 * B_ia, the component along the G=0-like eigenvector X_1 of V^cut(0) by the
 * q->0 limit sqrt(4 pi/Omega) (p_ia.q_hat)/D / sqrt(v_1) (Sec. III B, Eq.
 * dielectric_func_gamma as a Gram form); the result, screened with V^cut(0),
 * gives W^cut(0).
 * chi_out: complex T [n_freq][N_aux][N_aux], Hermitian.
 * Errors: ERR_ARG (D <= 0: an unoccupied level below an occupied one, or a
 * non-finite eigenvalue; the eigenvalues are read on every call, one small
 * copy to the host, so new contents at the same address are checked too;
 * apply_gamma without preparation or with iq != 0). */
int lrigw_chi0(lrigw_ctx *ctx, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out);

/* q = 0 preparation (Sec. III B): dominant eigenpair (X_1, v_1) of the
 * truncated Coulomb matrix Vcut0 (complex128 [N_aux][N_aux], Hermitian PD),
 * by power iteration on the device, X_1 scaled so its largest-magnitude
 * component is real positive; p: complex128 [N_k][n_occ][n_bands-n_occ],
 * momentum elements p_ia(k).q_hat; omega_cell: cell volume (bohr^3).
 * The context keeps X_1, v_1 and the pointer p (which must stay valid).
 * Errors: ERR_NOCONV (no dominant eigenvalue within 5000 iterations). */
int lrigw_gamma_prepare(lrigw_ctx *ctx, const void *Vcut0, const void *p, double omega_cell);

/* Screening (Eqs. symm_dielec_func and screened_W_matr), correlation part:
 *   W^c = V^{1/2} (eps~^{-1} - I) V^{1/2},  eps~ = I - V^{1/2} chi V^{1/2},
 * computed with the Cholesky factor V = L L^H in place of V^{1/2} (W is
 * unchanged by that substitution) and eps~^{-1} - I = -eps~^{-1}(eps~ - I)
 * (no cancellation at weak screening), all in FP64.
 * chi: complex T [n_freq][N_aux][N_aux] (lrigw_chi0 output); V: complex128
 * [N_aux][N_aux] (V(q), or V^cut(0) at iq == 0).  Wc_out: complex T, same
 * shape as chi.  info (host, may be NULL): -1, or the first frequency index
 * whose eps~ was not positive definite, or -2 if V was not.
 * Vcut: complex128 [N_aux][N_aux] truncated Coulomb matrix V^cut(q) (Sec. III
 * B, Eq. cut_coulomb_pot), or NULL (= V).  It replaces V in the numerator
 * only, W^c = V^cut^{1/2} (eps~^{-1} - I) V^cut^{1/2} with eps~ from the full
 * V, both roots the Hermitian ones: computed as T (eps~_L^{-1} - I) T^H with
 * T = V^cut^{1/2} V^{1/2} L^{-H}, the roots by a fixed number of coupled
 * Newton-Schulz steps on the device (exact to rounding for
 * |V|_F / lambda_min(V) up to 1e10; about 2 x 108 FP64 N_aux^3 GEMMs per
 * call).  A workspace of 13 N_aux^2 complex128 is allocated at the first such
 * call and kept by the context.
 * Errors: ERR_NOT_HPD, ERR_OOM. */
int lrigw_screen(lrigw_ctx *ctx, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info);

/* Correlation self-energy, Eq. GW_selfe_element with W -> W^c and w_q = 1/N_q,
 * folded onto w' > 0 (W^c is even in w'):
 *   sigma_acc[k][n][i] += -1/(pi N_q) sum_m sum_j g_j X_nm(k,q,w_j) a/(a^2 + w_j^2),
 *   a = i w_i + mu - e_m(k-q),  X_nm = sum_{mu nu} x^mu_nm W^c_{mu nu}(w_j) conj(x^nu_nm).
 * x: slice-1 output of lrigw_build_M for this iq; Wc: lrigw_screen output;
 * eig: FP64 [N_k][n_bands]; sigma_acc: complex128 [N_k][n_qp][n_freq],
 * accumulated (zero it before the first q). */
int lrigw_sigma_c(lrigw_ctx *ctx, int iq, const void *x, const void *Wc, const double *eig, void *sigma_acc);

/* Exchange self-energy: the bare-Coulomb term of Eq. GW_selfe_element
 * (W_0 = V + W^c).  V is static, and with the equal-time convergence factor
 * of the exchange term the frequency integral keeps the occupied bands:
 *   sigma_x[k][n] += -1/N_q sum_{m occ} sum_{mu nu} x^mu_nm V_{mu nu}(q) conj(x^nu_nm)
 * (the pairing of lrigw_sigma_c with W^c -> V; real since V is Hermitian),
 * computed in FP64 (the pairs are widened from the compute type).
 * xo: slice-2 output of lrigw_build_M for this iq; V: complex128
 * [N_aux][N_aux], V(q) (V(0) the truncated matrix of Sec. III B, as passed
 * to lrigw_screen); sigma_x: FP64 [N_k][n_qp] on the device, accumulated
 * (zero it before the first q).  A workspace of 2 * N_k*n_qp*n_occ*N_aux
 * complex128 is allocated at the first call and kept by the context.
 * Errors: ERR_ARG (iq out of range, NULL), ERR_OOM. */
int lrigw_sigma_x(lrigw_ctx *ctx, int iq, const void *xo, const void *V, double *sigma_x);

/* Sigma^x over every q: sigma_x (FP64 [N_k][n_qp], device) is set to the sum
 * over q of lrigw_sigma_x, with the pairs built by lrigw_build_M slice 2 into a
 * context buffer.  H: lrigw_lri_ft output; evec as for lrigw_lri_ft; V:
 * complex128 [N_k][N_aux][N_aux] (V[0] the truncated matrix).  Together with
 * the caller's V^xc it gives the static term of lrigw_qp:
 * e_static = sigma_x - V^xc.  Errors: ERR_ARG (NULL), ERR_OOM. */
int lrigw_sigma_x_pass(lrigw_ctx *ctx, const void *H, const void *evec, const void *V, double *sigma_x);

/* Pade continuation (Thiele continued fraction through n_par grid points
 * j*(n_freq-1)/(n_par-1) rounded half up) and the quasiparticle equation
 *   E = e_n + e_static_n + Re P_n(E - mu),  Z = 1/(1 - Re P_n'(E - mu)),
 * Newton from e_n + e_static_n (|dE| < 1e-10 Ha, <= 50 steps), else the sign
 * change of the residual nearest to the start within +-1 Ha (1 mHa scan) by
 * bisection.  sigma: complex128 [N_k][n_qp][n_freq]; eps_qp: FP64
 * [N_k][n_qp]; e_static: FP64 [N_k][n_qp] or NULL (zero).  e_qp, z: FP64
 * [N_k][n_qp] outputs.  info (host, may be NULL): number of (k,n) without a
 * root.  Returns WARN_QP_NOCONV / WARN_PADE_TRUNC when they occur. */
int lrigw_qp(lrigw_ctx *ctx, const void *sigma, const double *eps_qp, const double *e_static, int n_par,
             double *e_qp, double *z, int *info);

/* The continuation of lrigw_qp evaluated at real energies: out[e][k][n] =
 * P_{kn}(E[e][k][n] - mu), the same nodes and continued fraction (Sigma^c on
 * the real axis, e.g. for spectral functions or beside contour deformation).
 * sigma: complex128 [N_k][n_qp][n_freq]; E: FP64 [n_e][N_k][n_qp] absolute
 * energies (Ha); out: complex128 [n_e][N_k][n_qp]; all on the device.
 * Errors: ERR_ARG (NULL, n_par outside 1..64, n_e < 1). */
int lrigw_pade_eval(lrigw_ctx *ctx, const void *sigma, int n_par, int n_e, const double *E, void *out);

/* Whole path for one cell, q loop inside the library:
 *   for q: build_M(0), chi0 (gamma at q = 0 when p != NULL), screen (V[q]; V[0]
 *   is V^cut(0)), build_M(1), sigma_c;  then qp.
 * V: complex128 [N_k][N_aux][N_aux]; p: complex128 [N_k][n_occ][n_unocc] or
 * NULL (no q = 0 head/wings); H: lrigw_lri_ft output.  sigma: complex128
 * [N_k][n_qp][n_freq] output; e_qp, z: FP64 [N_k][n_qp].  q_first..q_last-1
 * restricts the q loop (0, N_k for all; QP only when all q were done).
 * Vcut: complex128 [N_k][N_aux][N_aux] truncated Coulomb matrices V^cut(q) for
 * the numerator of the screening at q != 0 (lrigw_screen), or NULL (V^cut =
 * V); Vcut[0] is not read (V[0] is V^cut(0), used in both places at q = 0).
 * The buffers for M, chi0 and W^c are owned by the context.  The Cholesky
 * factors of V(q) (and the V^cut factors) of q_first..q_last-1 are computed
 * once per call, batched.  Without graph capture, a surrogate or a direction
 * average, the q are screened in groups of up to 8 (as many as 8 GiB of
 * responses, W^c and FP64 workspace allow; the context keeps those buffers),
 * each group's screening beside the next group's responses. */
int lrigw_g0w0(lrigw_ctx *ctx, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
               const void *p, double omega_cell, const double *e_static, int n_par, int q_first, int q_last,
               void *sigma, double *e_qp, double *z, int *info);

/* Average the q -> 0 screening over directions of approach.  The head and
 * wings of Eq. dielectric_func_gamma depend on the direction q_hat along which
 * q -> 0 (Sec. III B); the paper gives no averaging scheme.  With n_dir > 0,
 * the whole passes (lrigw_g0w0, the batched graph, lrigw_sigma_cd_pass,
 * lrigw_g0w0_cd) take W^c(0) = sum_d weights[d] W^c(0; q_hat_d).  Each term is
 * the exact q = 0 response with p . q_hat_d and its screening, on the
 * context's stream; the surrogate is not used at q = 0.  The p argument of
 * those calls must still be non-NULL (it selects the q = 0 treatment).
 * p_dirs: device complex128 [n_dir][N_k][n_occ][n_unocc], p_ia(k) . q_hat_d.
 * It stays owned by the caller and must outlive the passes.  weights: host
 * double[n_dir], copied.  A set closed under q_hat -> -q_hat (e.g. the six
 * Cartesian half-axes, equal weights) removes the wing terms from W^c(0), and
 * with them the difference between Sigma^c(k) and Sigma^c(-k).  n_dir = 0
 * returns to the single direction.  Errors: ERR_ARG (n_dir outside 0..64,
 * NULL, non-finite weight). */
int lrigw_set_gamma_directions(lrigw_ctx *ctx, int n_dir, const void *p_dirs, const double *weights);

/* ---- Sigma^c at real energies by contour deformation (the alternative to
 * analytic continuation named in Sec. II A, after Eq. chi_0_realspace).
 *
 * Moving the real-axis frequency integral onto the imaginary axis leaves two
 * terms, with z = E - e_m(k-q) and X_nm(w) = x^T W^c(q,w) conj(x) the pair
 * weight of Eq. GW_selfe_element:
 *   Sigma^c_n(k,E) = 1/N_q sum_q sum_m [ -(1/pi) int_0^inf X_nm(iw) z/(z^2+w^2) dw
 *                                        + theta_m(E) X_nm(|z|) ]
 * The first is the imaginary-axis integral; the second collects the residues
 * of the Green-function poles passed over.  theta = +1 for an unoccupied m
 * below E, -1 for an occupied m above E, half of that at E = e_m, else 0.
 *
 * W^c on the real axis is formed below the smallest transition energy D_min
 * only.  There the response weight is 2D/(D^2 - w^2), chi~ is Hermitian and
 * eps~ positive definite.  This serves states near the band edges, whose
 * residues come from levels between mu and E.
 *
 * Discretisation:
 *  - Real planes: the uniform grid w_r = r h, r < n_r.  X between nodes is
 *    the 4-point Lagrange interpolant, with the stencil reflected at w = 0.
 *  - Imaginary-axis integral: the response grid, with X(0) (the first real
 *    plane) subtracted and its integral (pi/2) sgn(z) X(0) added in closed
 *    form.
 *  - A residue frequency above (n_r - 1) h makes that output NaN. */

/* Define the real grid w_r = r omega_max/(n_r-1).
 * eta = 0: 4 <= n_r <= n_freq planes below the smallest transition energy
 *   (exact, Hermitian W^c); allocates the context's real-axis buffers
 *   (4 n_r N_aux^2 complex of the compute type, n_r N_k n_qp n_bands doubles).
 * eta > 0: the broadened grid for every state, 4 <= n_r <= 65536 nodes at any
 *   height: W^c is taken at w_r + i eta (the poles of the time-ordered W^c
 *   broadened by eta; the grid step should resolve eta, e.g. eta/4).  The
 *   response of each node is the Re-weight plane plus i times the Im-weight
 *   plane of 2D/(D^2 - (w_r + i eta)^2); eps~ is then not Hermitian and is
 *   solved through its normal equations (E^H E) X = E^H D on the Cholesky
 *   path; the residues use Re X_nm, the quadratic form of the Hermitian part
 *   of W^c, which is what Re Sigma^c takes.  Used by lrigw_sigma_cd_pass,
 *   lrigw_g0w0_cd and lrigw_qp_cd (in chunks of n_freq/2 nodes, on the
 *   context stream alone; not with the direction average at q = 0); the
 *   single-q calls lrigw_chi0_real, lrigw_screen_real and lrigw_sigma_cd
 *   return ERR_ARG with it.  Allocates n_r N_k n_qp n_bands doubles.
 * Waits for the stream.  Errors: ERR_ARG (n_r, omega_max or eta out of
 * range; eta > 0 with n_freq < 2), ERR_OOM. */
int lrigw_set_real_grid(lrigw_ctx *ctx, int n_r, double omega_max, double eta);

/* chi~(q, w_r) at the n_r real frequencies: as lrigw_chi0 (same M, eig,
 * apply_gamma and output layout [n_r][N_aux][N_aux]), weight 2D/(D^2 - w^2).
 * Errors: ERR_ARG (no real grid, or omega_max >= the smallest transition
 * energy of eig, where the response has a pole), as lrigw_chi0 otherwise. */
int lrigw_chi0_real(lrigw_ctx *ctx, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out);

/* W^c(q, w_r) from lrigw_chi0_real's output: lrigw_screen over n_r planes
 * (Vcut as there). */
int lrigw_screen_real(lrigw_ctx *ctx, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info);

/* Contribution of q to Sigma^c_n(k, E) at n_e (1..4) sets of real energies.
 * x: slice-1 output of lrigw_build_M; Wc: lrigw_screen output (n_freq
 * planes); Wr: lrigw_screen_real output (n_r planes); E: FP64 [n_e][N_k][n_qp]
 * absolute energies (Ha) on the device; sigma_e: FP64 [n_e][N_k][n_qp],
 * accumulated.  Pair weights in the compute type, the combination in FP64.
 * Errors: ERR_ARG (NULL, iq out of range, no real grid, n_e outside 1..4). */
int lrigw_sigma_cd(lrigw_ctx *ctx, int iq, const void *x, const void *Wc, const void *Wr, const double *eig, int n_e,
                   const double *E, double *sigma_e);

/* lrigw_sigma_cd summed over every q.  The per-q response and W^c come from
 * the exact response on both grids, with the q = 0 head and wings when p !=
 * NULL.  Arguments are as for lrigw_g0w0 (V^cut included); sigma_e is set (not accumulated).
 * n_bad (host, may be NULL) receives the number of NaN outputs.
 * Returns WARN_CD_RANGE when there are any.  Screens q on the context's second
 * stream while the responses of q+1 are built (as lrigw_g0w0) and waits for
 * the stream at the end; not for graph capture.  Errors: ERR_ARG (NULL, no
 * real grid, n_e outside 1..4, p without omega_cell > 0, called while the
 * context captures a graph), ERR_NOT_HPD (a screening failed). */
int lrigw_sigma_cd_pass(lrigw_ctx *ctx, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                        const void *p, double omega_cell, int n_e, const double *E, double *sigma_e, int *n_bad);

/* Linearised quasiparticle energies from contour deformation:
 *   Sigma^c at e_n - delta, e_n, e_n + delta (e_n the band energies of the QP bands),
 *   E_n = e_n + Z (Sigma^c(e_n) + e_static_n),
 *   Z = 1 / (1 - (Sigma^c(e_n + delta) - Sigma^c(e_n - delta)) / (2 delta)).
 * sigma3: FP64 [3][N_k][n_qp] output or NULL; e_qp, z: FP64 [N_k][n_qp]
 * outputs; e_static may be NULL.  Returns WARN_CD_RANGE as lrigw_sigma_cd_pass;
 * states with a NaN among their three values get NaN energies.  Errors: as
 * lrigw_sigma_cd_pass, and ERR_ARG for delta <= 0. */
int lrigw_g0w0_cd(lrigw_ctx *ctx, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                  const void *p, double omega_cell, const double *e_static, double delta, double *sigma3, double *e_qp,
                  double *z, int *n_bad);

/* Quasiparticle energies from contour deformation by Newton steps on
 *   f(E) = E - e_n - e_static_n - Sigma^c(E),  E_0 = e_n,
 *   E <- E + Z (e_n + e_static_n + Sigma^c(E) - E),
 *   Z = 1 / (1 - (Sigma^c(E + delta) - Sigma^c(E - delta)) / (2 delta)),
 * n_iter (1..64) steps, each one whole contour-deformation pass at the three
 * energies of every state (n_iter = 1 is lrigw_g0w0_cd).  warm = 0 starts
 * from E_0 = e_n; warm = 1 continues from the energies e_qp holds on entry
 * (a call of n steps after one of m gives what one call of m + n steps
 * gives).  With the broadened grid (lrigw_set_real_grid, eta > 0) every state
 * is evaluated.  Arguments and errors as lrigw_g0w0_cd (ERR_ARG also for warm
 * outside 0..1); sigma3 holds the last pass's three values, z the Z of the
 * last step. */
int lrigw_qp_cd(lrigw_ctx *ctx, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                const void *p, double omega_cell, const double *e_static, double delta, int n_iter, int warm,
                double *sigma3, double *e_qp, double *z, int *n_bad);

/* ---- Learned frequency surrogate of the response (a form the paper does not
 * have; it evaluates Eq. chi0_matrix at every frequency of the grid).
 *
 * Per q the response is computed exactly at n_anchor anchor indices
 * j (n_freq-1)/(n_anchor-1) (rounded half up) and at one held-out index midway
 * between the two middle anchors; at every other index t it is predicted as
 *   chi(w_t) = sum_l C[l][t] chi(w_l) + U R_t U^H,
 * where C is a least-squares interpolation rule for the transition kernel
 * 2D/(D^2 + w^2) over D in [d_lo, d_hi] (256 log-spaced D, anchor columns
 * scaled to unit norm, ridge 1e-12), U (N_aux x rank) is an orthonormal basis
 * of the dominant eigenspace of -chi(w_anchor0) (4 block subspace-iteration
 * products from the caller's start block, Cholesky QR after each), and R_t is
 * the rule's residual on the rank x rank projection U^H chi U, predicted by a
 * network from the anchor values of each of its rank^2 real series (Re P_ij
 * for i <= j, Im P_ij for i > j) scaled by s = sign(a_0) |a|:
 *   h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3,
 * x = a/s (n_anchor inputs), y = residual/s at the n_out non-anchor indices.
 * Parameters: FP32 flat vector W1 [n_anchor][H], b1 [H], W2 [H][H], b2 [H],
 * W3 [H][n_out], b3 [n_out]; the products use the BF16-rounded copy with FP32
 * activations and accumulation.  If the relative Frobenius error of the
 * prediction at the held-out index exceeds `threshold`, every other index of
 * that q is recomputed exactly (decided on the device).  The surrogate serves
 * every context with the same N_aux, n_freq and x0 as the one it was created
 * with, and runs on that context's stream. */
typedef struct lrigw_surrogate lrigw_surrogate;

/* init_params: device FP32 [n_params] (see lrigw_surrogate_info); start:
 * device FP64 [N_aux][rank] (real); row_capacity: training rows to reserve
 * (rank^2 per added q).  Errors: ERR_ARG (n_anchor outside 4..16,
 * n_freq < n_anchor + 2, rank > N_aux or > 256, d_hi <= d_lo or d_lo <= 0),
 * ERR_OOM. */
int lrigw_surrogate_create(lrigw_ctx *ctx, int rank, int n_anchor, int hidden, double d_lo, double d_hi,
                           long long row_capacity, const float *init_params, const double *start,
                           lrigw_surrogate **out);
int lrigw_surrogate_destroy(lrigw_surrogate *sg);
/* ints (host, 6): n_anchor, n_out, held-out grid index, its position among
 * the n_out non-anchor indices, rank, hidden; n_params (host). */
int lrigw_surrogate_info(const lrigw_surrogate *sg, int *ints, long long *n_params);
/* The rule C (device FP64 [n_anchor][n_out]). */
int lrigw_surrogate_rule(const lrigw_surrogate *sg, double *C);
/* Copy the FP32 parameters out (get) and/or replace them (set; resets Adam). */
int lrigw_surrogate_params(lrigw_surrogate *sg, float *get, const float *set);
/* The basis U (device complex128 [N_aux][rank]) of chi_a0 (complex T
 * [N_aux][N_aux] of ctx's precision). */
int lrigw_surrogate_basis(lrigw_surrogate *sg, lrigw_ctx *ctx, const void *chi_a0, void *U_out);
/* Append the rank^2 training rows of one q from the exact response chi
 * (complex T [n_freq][N_aux][N_aux]): x = scaled anchor values, target = the
 * rule's residual at the non-anchor indices in units of s.  Synchronous.
 * Errors: ERR_ARG (capacity), ERR_NOT_HPD (basis rank-deficient). */
int lrigw_surrogate_add(lrigw_surrogate *sg, lrigw_ctx *ctx, const void *chi);
/* Row count (host) and rows first..first+count-1 (device FP32 x
 * [count][n_anchor], y [count][n_out]; either may be NULL). */
int lrigw_surrogate_rows(lrigw_surrogate *sg, long long *n_rows, float *x, float *y, long long first, long long count);
/* Network output y (device FP32 [n_rows][n_out]) for inputs x [n_rows][n_anchor]. */
int lrigw_surrogate_forward(lrigw_surrogate *sg, const float *x, int n_rows, float *y);
/* Mean-squared loss (device float[1]) and its gradient (device FP32
 * [n_params]) for rows x, y; no update. */
int lrigw_surrogate_grad(lrigw_surrogate *sg, const float *x, const float *y, int n_rows, float *loss, float *grad);
/* `steps` Adam steps (beta 0.9/0.999, eps 1e-8, learning rate lr) on batches
 * of the stored rows: step s uses rows order[s*batch .. s*batch+batch-1]
 * (device int32, order_len >= steps*batch).  loss_hist: device float[steps]
 * or NULL. */
int lrigw_surrogate_train(lrigw_surrogate *sg, int steps, int batch, double lr, const int *order, long long order_len,
                          float *loss_hist);
/* Response of one q with the surrogate (arguments as lrigw_chi0). */
int lrigw_chi0_surrogate(lrigw_ctx *ctx, lrigw_surrogate *sg, int iq, const void *M, const double *eig, int apply_gamma,
                         double threshold, void *chi_out);
/* Make lrigw_g0w0 use the surrogate for every q (sg = NULL: exact). */
int lrigw_set_surrogate(lrigw_ctx *ctx, lrigw_surrogate *sg, double threshold);
/* Calls so far (host), fallbacks (host int), and the held-out errors of the
 * first max_errors calls (host FP64).  Synchronises the stream. */
int lrigw_surrogate_stats(lrigw_surrogate *sg, long long *n_calls, int *n_fallback, double *errors, int max_errors);
int lrigw_surrogate_reset_stats(lrigw_surrogate *sg);

/* ---- Batched form: several cells (uneven basis and auxiliary sizes, each
 * with its own context and precision) in one hipGraph.  The graph holds the
 * whole pass of every cell (lrigw_g0w0's q loop and QP step; cells on
 * separate streams inside the graph); lrigw_batch_run replays it with one
 * launch.  Everything that needs the host (gap check, q = 0 preparation,
 * buffers, tuning) is done by lrigw_batch_create.  With autotune != 0 the
 * response kernel of every cell is timed on one q over its tile choices
 * (frequencies per workgroup, K split count) and the fastest is kept.
 * The arrays a cell names must stay valid while the batch exists; inputs may
 * change between runs (same addresses).  The eigenvalues are checked for a
 * gap (every unoccupied level above every occupied one) at create only: the
 * graph does not re-check them, so new eigenvalues must keep that order. */
typedef struct {
  lrigw_ctx *ctx;                 /* one context per cell */
  const void *H, *evec;           /* lrigw_lri_ft output, eigenvectors (device) */
  const double *eig;              /* FP64 [N_k][n_bands] (device) */
  const void *V, *Vcut, *p;       /* as lrigw_g0w0; Vcut and p may be NULL */
  double omega_cell;
  const double *e_static;         /* FP64 [N_k][n_qp] or NULL */
  int n_par;                      /* Pade points (1..64) */
  void *sigma;                    /* complex128 [N_k][n_qp][n_freq] output */
  double *e_qp, *z;               /* FP64 [N_k][n_qp] outputs */
} lrigw_batch_cell;
typedef struct lrigw_batch lrigw_batch;

/* hip_stream must be a created stream (not the legacy default stream).  A
 * surrogate attached with lrigw_set_surrogate is captured too (its call
 * statistics then count the capture, not the replays).
 * Errors: ERR_ARG (NULL arrays, a context used twice), ERR_NOT_HPD /
 * ERR_NOCONV from the q = 0 preparation, ERR_HIP (capture). */
int lrigw_batch_create(lrigw_batch **out, int n_cells, const lrigw_batch_cell *cells, int autotune, void *hip_stream);
/* One launch of the captured graph on hip_stream (asynchronous). */
int lrigw_batch_run(lrigw_batch *b);
/* After a run (synchronises): status[3*i + 0] = first q of cell i whose V or
 * eps~ was not positive definite, or -1; [3*i + 1] = QP equations without a
 * root; [3*i + 2] = truncated Pade fits. */
int lrigw_batch_status(lrigw_batch *b, int *status);
/* The tuned tile choice of a cell and its measured time (ms, -1 untuned). */
int lrigw_batch_tuning(const lrigw_batch *b, int cell, int *nw, int *splits, double *ms);
int lrigw_batch_graph_nodes(const lrigw_batch *b, long long *n_nodes);
int lrigw_batch_destroy(lrigw_batch *b);

/* Tile autotuner for one context (the same one lrigw_batch_create runs per
 * cell): times the response kernel on one q over its tile choices
 * (frequencies per workgroup, K splits, LDS row padding) and, in the split
 * forms, the self-energy kernel over its variants (frequencies per workgroup,
 * W prefetch, wave tile, LDS row padding, x tile resident in LDS), and keeps
 * the fastest for the context's later calls; candidates are tried in a fixed
 * order and a later one replaces the best so far only if it is at least 2%
 * faster, so near-ties resolve the same way each time (the K split count
 * changes the order of the FP32 sums).
 * H, evec, eig as lrigw_g0w0.  Outputs (host, may be NULL): the chosen
 * response tiles, the self-energy variant (0..13) and the response time of one
 * q (ms).
 * Synchronous. */
int lrigw_tune(lrigw_ctx *ctx, const void *H, const void *evec, const double *eig, int *nw, int *splits,
               int *sigma_variant, double *ms);

/* Set the tile choices lrigw_tune would pick, explicitly: nw = frequencies per
 * response workgroup (the form's default or its alternative: 4/2 in the FP32
 * and split forms, 2/1 in FP64), splits = K splits, 1..max(1, K/64), K =
 * N_k n_occ n_unocc (in the split forms at least ceil(K/4096), so no
 * workgroup sums more than 4096 rows in FP32; splits beyond what the
 * context's partial-tile buffer of at most 3 GiB holds run in batches whose
 * results are added up in the output), pad = LDS row padding of the split-form response kernel (8
 * or 16), sigma_variant = split-form self-energy kernel variant (0..13; 7 to
 * 13, the resident-tile form with 8 or 4 waves and LDS rows padded by 8 or
 * 16, (11, 12) the per-tile sum taking x from global memory, or (13) 8 waves
 * with the frequencies in four sets instead of eight, twice as many per
 * workgroup, need the two-part FP16 split, N_aux <= 288 and at most 32
 * frequencies).
 * Errors: ERR_ARG for a choice outside these sets or a variant the cell does
 * not admit. */
int lrigw_set_tiles(lrigw_ctx *ctx, int nw, int splits, int pad, int sigma_variant);

/* The current tile choices (host outputs, any may be NULL) and the number of
 * self-energy kernel variants (valid ones are 0..n_variants-1). */
int lrigw_get_tiles(const lrigw_ctx *ctx, int *nw, int *splits, int *pad, int *sigma_variant, int *n_variants);

/* Per-kernel device time (ms, HIP events on the stream each stage runs on)
 * accumulated since the last reset, for the named stages "lri_ft", "build_M",
 * "chi0" (with its parts "chi0_split" and "chi0_mfma"), "screen", "sigma_c"
 * (with "sigma_split" and "sigma_mfma") and "qp".  lrigw_set_timing(ctx, on):
 * on = 0 records nothing, 1 every stage, 2 only the two MFMA kernel stages
 * "chi0_mfma" and "sigma_mfma" (two events per launch, nothing recorded
 * between the other kernels of a pass); other values return LRIGW_ERR_ARG.
 * lrigw_stage_ms returns -1.0 for an unknown stage. */
int lrigw_set_timing(lrigw_ctx *ctx, int on);
double lrigw_stage_ms(lrigw_ctx *ctx, const char *stage, long long *launches);
void lrigw_reset_timing(lrigw_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LRIGW_H */
