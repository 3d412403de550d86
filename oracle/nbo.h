/*
 * nbo.h -- CPU oracle for the bulb-model radial stepper (plain FP64 C).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference that the HIP
 * path is checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.
 *
 * Physics (paper, Sec. 2): every beam is labelled by species s (neutrino / antineutrino,
 * optionally every initial flavour), emission bin u_j = sin^2(theta_R) and energy bin
 * E_k.  Its flavour state evolves along the radius r by
 *     i cos(theta) d/dr psi = H psi,   H = H_vac + H_mat + H_nunu          (Eq. eom)
 * with H_nunu built from two energy/angle moments of all beams (Eqs. Hnu and F).
 * The integrator is a Lie-group Runge-Kutta method of order 4 (classical RK4 tableau,
 * Munthe-Kaas 1999) whose exponential map is the exact one-step propagator of Eq. U.
 *
 * All entry points return 0 on success and a negative code on failure.
 */
#ifndef NBO_H
#define NBO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { NBO_OK = 0, NBO_EINVAL = -1, NBO_ENUMERIC = -5, NBO_ESTEP = -7 };

typedef struct {
  int32_t n_flavor;     /* 2 or 3 */
  int32_t n_energy;     /* N_E energy bins, equal width over [e_min, e_max] */
  int32_t n_u;          /* N_u emission bins, equal width in u = sin^2 theta_R over [0,1] */
  int32_t ne_power;     /* n_e(r) = n0 (R/r)^ne_power; 3 for the bulb, 0 = constant density */
  int32_t renorm;       /* 1: renormalise every beam after every step */
  int32_t integrator;   /* 0: RKMK4 (exact exponentials); 1: plain RK4 on the ODE */
  int32_t species4;     /* 0: track nu_e- and anti-nu_e-born beams only;
                           1: track every initially populated flavour explicitly */
  int32_t n_phi;        /* 0: the bulb model (axial symmetry); >= 1: the extended bulb
                           model with n_phi azimuthal bins of equal width over [0, 2pi) */
  int64_t n_steps;
  double e_min_mev, e_max_mev, r_nu_km, r_start_km, r_end_km;
  double lum_erg_s[3];  /* nu_e, anti-nu_e, nu_x (= every heavy flavour and antiflavour) */
  double temp_mev[3];
  double dm2_ev2[2];    /* 2f: [0] = dm^2;  3f: dm^2_21, dm^2_31 */
  double theta[3];      /* 2f: [0] = theta_v;  3f: theta_12, theta_13, theta_23 */
  double delta_cp;      /* must be 0 */
  double n0_cm3;
  double lum_xbar_erg_s, temp_xbar_mev;  /* anti-nu_x (= each heavy antiflavour); temp 0:
                                            the nu_x values of lum_erg_s[2], temp_mev[2] */
} nbo_params;

typedef struct nbo_model nbo_model;

int  nbo_create(const nbo_params *p, nbo_model **out);
void nbo_destroy(nbo_model *m);
int  nbo_set_threads(int n);                     /* OpenMP threads (0 = default) */
int  nbo_get_threads(void);                      /* threads a parallel region will use */
int64_t nbo_n_beams(const nbo_model *m);
int  nbo_n_species(const nbo_model *m);
int  nbo_state_comps(const nbo_model *m);         /* 3 (2f Bloch vector) or 6 (3f psi) */
int  nbo_reset(nbo_model *m);
int  nbo_step(nbo_model *m, int64_t n);
int64_t nbo_step_index(const nbo_model *m);
/* Re rho_ee of every beam, layout [species][n_u][n_phi][n_energy] (n_phi = 1 for the
 * bulb model). */
int  nbo_read_pee(const nbo_model *m, double *out);
/* State exchange: [comp][beam] planes, beam = (s*n_u + j)*n_energy + k. */
int  nbo_get_state(const nbo_model *m, double *out);
int  nbo_set_state(nbo_model *m, const double *in, int64_t step);
/* Tables, for comparison with the HIP path's host set-up:
 * out[0..NE) = E_k, then weights [n_species][NE], then the per-energy vacuum terms
 * (2f: bx, bz per k; 3f: 6 per k), then scalars {lam0, kappa0, h, 2^-e1, 2^-e0, e1, e0}. */
int  nbo_tables(const nbo_model *m, double *out, int64_t cap);
/* Moments J0 (ncomp) and J1 (ncomp) of the current state at radius r (Eq. F). */
int  nbo_moments(const nbo_model *m, double r, double *j0, double *j1);
/* All moments as [4][ncomp]: J0, J1, and for the extended model J_sc, J_ss (else 0). */
int  nbo_moments4(const nbo_model *m, double r, double *jm);
/* Per-beam Hamiltonian for the four moments jm [4][ncomp] (layout as nbo_hamiltonian). */
int  nbo_hamiltonian4(const nbo_model *m, double r, const double *jm, double *out);
/* cos and sin of the azimuth of every azimuthal bin ([2][n_phi]); extended model only. */
int  nbo_phi_table(const nbo_model *m, double *out);
/* Per-beam Hamiltonian at radius r for given moments (2f: B vector, 3 per beam;
 * 3f: Hermitian matrix d0,d1,d2,Re/Im o01,o02,o12 = 9 per beam).  Not scaled by h/c. */
int  nbo_hamiltonian(const nbo_model *m, double r, const double *j0, const double *j1,
                     double *out);
/* Geometry: c_j(r) for every angle bin. */
int  nbo_cos_theta(const nbo_model *m, double r, double *out);

/* Primitives of the arithmetic specification (exported for the pin tests). */
void nbo_sincos(const double *x, int64_t n, double *s, double *c);
/* psi' = exp(-i K) psi up to a global phase; K = 9 reals (as above), psi = 6 reals. */
void nbo_exp3_apply(const double *k9, const double *psi6, double *out6);
/* P' = R(x) P: rotation of the Bloch vector P about x by |x|. */
void nbo_rotate(const double *x3, const double *p3, double *out3);
/* Exact fixed-point sum of n doubles scaled by 2^e, returned as a double (tests). */
double nbo_fixed_sum(const double *v, int64_t n, int e);
/* The fixed-point integer of each beam contribution: v ws rounded to the nearest integer,
 * ties to even (|v ws| <= 2^51). */
void nbo_fix_round(const double *v, const double *ws, int64_t n, int64_t *out);

/* Adaptive step-size control (RKMK4 steps with an embedded order-2 error estimate; see
 * nbo.c for the controller).  From step 0 to r_end; *accepted, *rejected and the step
 * length after the last decision (*h_last) are reported.  h_max <= 0: no cap.
 * Returns NBO_ESTEP if the step length underflows or max_attempts is exceeded. */
int  nbo_run_adaptive(nbo_model *m, double tol, double h_max, int64_t max_attempts,
                      int64_t *accepted, int64_t *rejected, double *h_last);

/* Error estimate of one step of length h from the current state (no state change). */
int  nbo_step_error(nbo_model *m, double h, double *E);

/* Separately coded single-angle solver (2 flavours): one emission bin at u = 1/2. */
int  nbo_single_angle_run(const nbo_params *p, double *pee_out /* [2][NE] */);

/* Reverse-mode adjoint of the whole radial integration (2 flavours, RKMK4).
 * Runs forward from the current state to n_steps, keeping the state every ckpt steps,
 * then backwards segment by segment (each segment recomputed from its checkpoint).
 * L = sum_b dl_dpee[b] Pee_b of the final state; dl_dpee = NULL takes the energy-integrated
 * loss dl_dpee[b] = dE/N_u.  grad[5] = dL/d{L_e, L_ebar, L_x, theta_v, n0}; *loss = L;
 * state_bar (NULL or [nb][3]) = dL/d(initial Bloch vectors).  The model ends at n_steps. */
int  nbo_adjoint(nbo_model *m, int32_t ckpt, const double *dl_dpee, double *grad, double *loss,
                 double *state_bar);


/* ---- plain mode (plain.c): the step evaluated straight from its definitions ----
 * Density matrices as full complex matrices, dense per-beam generators and commutators,
 * exponentials by Jacobi eigen-decomposition, plain FP64 sums, exact renormalisation;
 * it shares no arithmetic with the functions above.  Fixed-step RKMK4 only (integrator
 * must be 0).  Complex arrays are interleaved (re, im). */
typedef struct plain_model plain_model;
int  nbp_create(const nbo_params *p, plain_model **out);
void nbp_destroy(plain_model *m);
int64_t nbp_n_beams(const plain_model *m);
int64_t nbp_step_index(const plain_model *m);
int  nbp_reset(plain_model *m);
int  nbp_step(plain_model *m, int64_t n);
/* Re rho_ee of every beam, beam order as nbo_read_pee */
int  nbp_read_pee(const plain_model *m, double *out);
/* rho of every beam, [nb][n][n] complex */
int  nbp_get_rho(const plain_model *m, double *out);
int  nbp_set_rho(plain_model *m, const double *in, int64_t step);
/* moments of the current state at radius r, [4][n][n] complex: J0, J1, Jsc, Jss */
int  nbp_moments(const plain_model *m, double r, double *out);
/* Hamiltonian of every beam at radius r for the current state's moments, [nb][n][n] */
int  nbp_hamiltonian(const plain_model *m, double r, double *out);
/* exp(-i K) for a Hermitian n x n K (n = 2, 3), [n][n] complex in and out */
void nbp_expm(int n, const double *k, double *out);

#ifdef __cplusplus
}
#endif
#endif
