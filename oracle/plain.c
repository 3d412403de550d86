/*
 * plain.c -- the oracle's plain mode: the bulb-model radial step evaluated straight from
 * its definitions in FP64, with none of the restated arithmetic of nbo.c.
 *
 * TEST INFRASTRUCTURE ONLY (see nbo.h).  Nothing in the product path links this file.
 *
 * nbo.c follows an arithmetic specification that the HIP library repeats operation for
 * operation (so that the two agree bit for bit even where the bulb model amplifies
 * rounding); this file shares none of it.  It is the second, independent reference: the
 * HIP path and nbo.c are compared with it within a tolerance on inputs where the
 * discrete evolution is well conditioned.  What differs from nbo.c:
 *   - the state of a beam is its density matrix rho as a full n x n complex matrix
 *     (nbo.c: Bloch vector or wavefunction);
 *   - every generator is formed per beam as a dense matrix, F_i = -i (h/c) H, and the
 *     commutators of the Lie-group RK4 are dense matrix products (nbo.c: per-row
 *     constants and bilinear forms);
 *   - exp(Omega) of an anti-Hermitian Omega = -i K comes from the eigen-decomposition of
 *     K by the cyclic Jacobi method with complex (Hermitian) rotations,
 *     exp(Omega) = V diag(exp(-i lambda)) V^+, with libm's sin and cos (nbo.c: largest
 *     eigenvalue by Halley steps, a cofactor eigenvector, the 2x2 propagator on the
 *     orthogonal plane and its own sin/cos);
 *   - moments are plain FP64 sums, energy first within a row, rows in order (nbo.c: exact
 *     fixed-point sums);
 *   - renormalisation makes rho Hermitian with unit trace and rescales its traceless part
 *     to unit purity Tr rho^2 = 1, with a true square root (nbo.c: one Newton step);
 *   - no fma anywhere, and the full Hamiltonian (trace included) is used.
 * Tables are formed here as well, from the same formulas (they are the definitions).
 *
 * The physics, with the paper's equations:
 *   beams b = (s, j[, p], k): species s (nu / anti-nu, or every born flavour), emission
 *   bin u_j = sin^2(theta_R) (midpoints), azimuthal bin p (extended model), energy E_k
 *   (midpoints)                                                             (Sec. 3.2)
 *   rho~_b = rho_b (nu), -conj(rhobar_b) (anti-nu)                           (Eq. F)
 *   J0 = sum_b g_b rho~_b / c_b(r),  J1 = sum_b g_b rho~_b,  and in the extended model
 *   Jsc = sum_b g_b rho~_b s_b cos(phi_b) / c_b,  Jss (sin(phi_b)),
 *   with c_b(r) = sqrt(1 - u_j R^2/r^2), s_b(r) = sqrt(u_j) R / r and weights
 *   g_b = kappa0 du dE N f(E_k) [/ n_phi] (heavy-flavour-born states enter as -N_x f_x
 *   through unitarity when only electron-born beams are tracked)     (Eqs. Hnu, F, int-v)
 *   H_nunu,b = mu(r) [(J0 - c_b J1) - s_b (cos(phi_b) Jsc + sin(phi_b) Jss)],
 *   mu(r) = R^2 / (2 r^2)                                                    (Eq. Hnu)
 *   H_b = H_vac(E_k) + lam(r) E_ee + H_nunu,b           (nu)
 *   H_b = H_vac(E_k) - lam(r) E_ee - conj(H_nunu,b)     (anti-nu)            (Eq. eom)
 *   H_vac = (dm^2/4E) [[-cos 2t, sin 2t], [sin 2t, cos 2t]]  (2f);
 *   H_vac = U diag(0, dm21, dm31) U^T / 2E  (3f, real U = R23 U13 R12)       (Sec. 2)
 *   lam(r) = sqrt2 G_F n0 (R/r)^ne_power                                      (Sec. 2)
 *   one fixed step r_n -> r_{n+1} (stage radii r_n, r_n + h/2, r_n + h/2, r_{n+1}):
 *   F_i = -i (h / c_b(r_i)) H_b(r_i, J(Y_i))       (Eq. U: the path step is dr / cos)
 *   Y_1 = rho_n,  Y_i = e^{Omega_i} rho_n e^{-Omega_i},  Omega_2 = F1/2,
 *   Omega_3 = F2/2 - [F1,F2]/8,  Omega_4 = F3,
 *   rho_{n+1} = e^{Theta} rho_n e^{-Theta},  Theta = (F1 + 2F2 + 2F3 + F4)/6 - [F1,F4]/12
 *   (the classical RK4 tableau on the unitary group, Munthe-Kaas 1999).
 *
 * Pins (tests/test_oracle_plain.py): the Jacobi exponential against SciPy's expm, vacuum
 * and constant-density closed forms, the Hamiltonian against the direct beam-pair sum,
 * one step against dense SciPy matrices, fourth-order convergence, trace and purity
 * without renormalisation, the flux-weighted invariant, single angle = one angle bin,
 * tracked species = every flavour explicit, the extended model's axial-symmetry
 * consistency, and agreement with nbo.c on well-conditioned inputs.
 */
#include "nbo.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

/* ------------------------------------------------------------ constants (A5) */
#define P_GF_GEV2 1.1663787e-5        /* Fermi constant */
#define P_HBARC_GEV_CM 1.973269804e-14  /* hbar c */
#define P_HBARC_EV_KM 1.973269804e-10
#define P_C_CM_S 2.99792458e10
#define P_ERG_MEV 6.241509074460763e5
#define P_PI 3.14159265358979323846
/* Fermi-Dirac integrals int_0^inf x^n / (e^x + 1) dx: F2 = 3 zeta(3) / 2, F3 = 7 pi^4 / 120 */
#define P_ZETA3 1.2020569031595942854
#define P_F2 (1.5 * P_ZETA3)
#define P_F3 (7.0 * P_PI * P_PI * P_PI * P_PI / 120.0)

/* sqrt(2) G_F n_e as a wavenumber in km^-1 per cm^-3: sqrt2 G_F (hbar c)^3 / (hbar c)_km */
static double plain_sqrt2gf(void) {
  const double hc3 = P_HBARC_GEV_CM * P_HBARC_GEV_CM * P_HBARC_GEV_CM;
  return sqrt(2.0) * P_GF_GEV2 * hc3 / (P_HBARC_GEV_CM * 1.0e-5);
}

/* --------------------------------------------------------- small dense algebra */
typedef struct { zc a[3][3]; } mat;

static mat m_zero(void) { mat m; memset(&m, 0, sizeof m); return m; }
static mat m_mul(int n, const mat *A, const mat *B) {
  mat C = m_zero();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      zc s = 0.0;
      for (int l = 0; l < n; ++l) s += A->a[i][l] * B->a[l][j];
      C.a[i][j] = s;
    }
  return C;
}
static mat m_adj(int n, const mat *A) { /* conjugate transpose */
  mat C = m_zero();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C.a[i][j] = conj(A->a[j][i]);
  return C;
}
static mat m_lin(int n, zc a, const mat *A, zc b, const mat *B) { /* a A + b B */
  mat C = m_zero();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C.a[i][j] = a * A->a[i][j] + b * B->a[i][j];
  return C;
}
static mat m_comm(int n, const mat *A, const mat *B) { /* [A, B] */
  const mat AB = m_mul(n, A, B), BA = m_mul(n, B, A);
  return m_lin(n, 1.0, &AB, -1.0, &BA);
}

/* Eigen-decomposition K = V diag(lam) V^+ of a Hermitian K (n <= 3) by the cyclic Jacobi
 * method: each rotation in the (p, q) plane first turns the phase of K_pq away
 * (D = diag(1, e^{-i arg K_pq}) on p, q) and then applies the real symmetric Jacobi
 * rotation that zeroes the now real entry (tan 2 theta = 2 |K_pq| / (K_qq - K_pp), the
 * smaller root t = tan theta); sweeps over all pairs until the off-diagonal part is below
 * 1e-17 of the matrix norm (at most 30 sweeps; the method converges quadratically). */
static void jacobi_herm(int n, const mat *K, mat *V, double lam[3]) {
  mat A = *K;
  /* Hermitian part, so that rounding in K cannot leave an imaginary diagonal */
  for (int i = 0; i < n; ++i) {
    A.a[i][i] = creal(A.a[i][i]);
    for (int j = i + 1; j < n; ++j) {
      const zc x = 0.5 * (A.a[i][j] + conj(A.a[j][i]));
      A.a[i][j] = x;
      A.a[j][i] = conj(x);
    }
  }
  *V = m_zero();
  for (int i = 0; i < n; ++i) V->a[i][i] = 1.0;
  double fro = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) fro += creal(A.a[i][j] * conj(A.a[i][j]));
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += 2.0 * creal(A.a[p][q] * conj(A.a[p][q]));
    if (!(off > 1e-34 * fro)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double g = cabs(A.a[p][q]);
        if (g == 0.0) continue;
        const zc e = A.a[p][q] / g;             /* e^{i arg K_pq} */
        const double app = creal(A.a[p][p]), aqq = creal(A.a[q][q]);
        const double th = (aqq - app) / (2.0 * g);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* G = D R: G_pp = c, G_pq = s, G_qp = -s conj(e), G_qq = c conj(e), the identity
         * elsewhere.  A <- G^+ A G and V <- V G touch only rows and columns p, q. */
        const zc gpp = c, gpq = s, gqp = -s * conj(e), gqq = c * conj(e);
        for (int i = 0; i < n; ++i) {   /* columns p, q of A G and of V G */
          const zc ap = A.a[i][p], aq = A.a[i][q];
          A.a[i][p] = ap * gpp + aq * gqp;
          A.a[i][q] = ap * gpq + aq * gqq;
          const zc vp = V->a[i][p], vq = V->a[i][q];
          V->a[i][p] = vp * gpp + vq * gqp;
          V->a[i][q] = vp * gpq + vq * gqq;
        }
        for (int i = 0; i < n; ++i) {   /* rows p, q of G^+ (A G) */
          const zc tp = A.a[p][i], tq = A.a[q][i];
          A.a[p][i] = conj(gpp) * tp + conj(gqp) * tq;
          A.a[q][i] = conj(gpq) * tp + conj(gqq) * tq;
        }
        A.a[p][q] = 0.0;
        A.a[q][p] = 0.0;
        for (int i = 0; i < n; ++i) A.a[i][i] = creal(A.a[i][i]);
      }
  }
  for (int i = 0; i < n; ++i) lam[i] = creal(A.a[i][i]);
}

/* exp(Omega) for anti-Hermitian Omega: K = i Omega is Hermitian, K = V diag(lam) V^+ and
 * exp(Omega) = exp(-i K) = V diag(exp(-i lam)) V^+. */
static mat expm_antiherm(int n, const mat *Om) {
  mat K = m_zero();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) K.a[i][j] = I * Om->a[i][j];
  mat V;
  double lam[3];
  jacobi_herm(n, &K, &V, lam);
  mat D = m_zero();
  for (int i = 0; i < n; ++i) D.a[i][i] = cos(lam[i]) - I * sin(lam[i]);
  const mat Vh = m_adj(n, &V);
  const mat T = m_mul(n, &D, &Vh);
  return m_mul(n, &V, &T);
}

/* e^{Omega} rho e^{-Omega} = E rho E^+ with E = exp(Omega) */
static mat conjugate(int n, const mat *Om, const mat *rho) {
  const mat E = expm_antiherm(n, Om);
  const mat Eh = m_adj(n, &E);
  const mat T = m_mul(n, rho, &Eh);
  return m_mul(n, &E, &T);
}

/* Hermitian, unit trace, unit purity: rho <- (rho + rho^+)/2, then rho = I/n + s rho0 with
 * rho0 the traceless part and s chosen so that Tr rho^2 = 1/n + s^2 Tr rho0^2 = 1. */
static void renormalise(int n, mat *rho) {
  mat H = m_zero();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) H.a[i][j] = 0.5 * (rho->a[i][j] + conj(rho->a[j][i]));
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += creal(H.a[i][i]);
  for (int i = 0; i < n; ++i) H.a[i][i] -= tr / n;
  double p2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) p2 += creal(H.a[i][j] * conj(H.a[i][j]));
  const double s = (p2 > 0.0) ? sqrt((1.0 - 1.0 / n) / p2) : 1.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) rho->a[i][j] = s * H.a[i][j] + ((i == j) ? 1.0 / n : 0.0);
}

/* ------------------------------------------------------------------- model */
struct plain_model {
  nbo_params p;
  int n;                   /* flavours */
  int ns;                  /* species rows */
  int anti[6], flav[6];    /* antiparticle flag and flavour of birth of each row */
  int64_t NE, NU, NP, nb;  /* energy, emission, azimuthal bins (NP = 1: bulb model) */
  int ext;                 /* extended bulb model */
  double dE, du, h, R, lam0;
  double *E, *g;           /* E[k]; g[s NE + k] */
  double *cphi, *sphi;
  mat *hvac;               /* [NE] */
  mat *rho, *Y;            /* [nb] */
  int64_t step;
};
typedef struct plain_model plain_model;

/* moments of one radius: J[0] = J0, J[1] = J1, J[2] = Jsc, J[3] = Jss */
typedef struct { mat J[4]; } moments_t;

static double fermi_dirac(double E, double T) {
  return E * E / (P_F2 * T * T * T * (exp(E / T) + 1.0));
}

static void beam_of(const plain_model *m, int64_t b, int *s, int64_t *j, int64_t *p, int64_t *k) {
  *k = b % m->NE;
  const int64_t row = b / m->NE;
  *p = row % m->NP;
  *j = (row / m->NP) % m->NU;
  *s = (int)(row / (m->NP * m->NU));
}
static double u_bin(const plain_model *m, int64_t j) { return (j + 0.5) / (double)m->NU; }
static double cos_theta(const plain_model *m, int64_t j, double r) {
  return sqrt(1.0 - u_bin(m, j) * (m->R / r) * (m->R / r));
}
static double sin_theta(const plain_model *m, int64_t j, double r) {
  return sqrt(u_bin(m, j)) * m->R / r;
}

int nbp_create(const nbo_params *p, plain_model **out) {
  *out = NULL;
  if (!p || (p->n_flavor != 2 && p->n_flavor != 3) || p->n_energy < 1 || p->n_u < 1 ||
      p->n_steps < 1 || !(p->r_start_km >= p->r_nu_km) || !(p->r_end_km > p->r_start_km) ||
      !(p->e_max_mev > p->e_min_mev) || !(p->e_min_mev > 0.0) || p->delta_cp != 0.0 ||
      p->ne_power < 0 || p->ne_power > 8 || !(p->r_nu_km > 0.0) || p->n_phi < 0 ||
      p->n_phi > 4096 || p->integrator != 0)
    return NBO_EINVAL;
  plain_model *m = (plain_model *)calloc(1, sizeof *m);
  m->p = *p;
  m->n = p->n_flavor;
  if (!p->species4) {
    m->ns = 2;
    m->anti[0] = 0; m->flav[0] = 0;
    m->anti[1] = 1; m->flav[1] = 0;
  } else {
    m->ns = 2 * m->n;
    for (int s = 0; s < m->ns; ++s) { m->anti[s] = s / m->n; m->flav[s] = s % m->n; }
  }
  m->ext = p->n_phi >= 1;
  m->NP = m->ext ? p->n_phi : 1;
  m->NE = p->n_energy;
  m->NU = p->n_u;
  m->nb = (int64_t)m->ns * m->NU * m->NP * m->NE;
  m->dE = (p->e_max_mev - p->e_min_mev) / m->NE;
  m->du = 1.0 / m->NU;
  m->h = (p->r_end_km - p->r_start_km) / p->n_steps;
  m->R = p->r_nu_km;
  m->lam0 = plain_sqrt2gf() * p->n0_cm3;
  /* nu-nu prefactor: sqrt2 G_F N / (2 pi R^2 c) per unit number luminosity N (s^-1), the
   * half-isotropic emission from the neutrinosphere (Eq. Hnu) */
  const double rcm = m->R * 1.0e5;
  const double kappa0 = plain_sqrt2gf() / (2.0 * P_PI * rcm * rcm * P_C_CM_S);
  m->E = (double *)malloc(sizeof(double) * m->NE);
  m->g = (double *)malloc(sizeof(double) * m->NE * m->ns);
  m->hvac = (mat *)malloc(sizeof(mat) * m->NE);
  m->cphi = (double *)malloc(sizeof(double) * m->NP);
  m->sphi = (double *)malloc(sizeof(double) * m->NP);
  m->rho = (mat *)malloc(sizeof(mat) * m->nb);
  m->Y = (mat *)malloc(sizeof(mat) * m->nb);
  if (!m->E || !m->g || !m->hvac || !m->cphi || !m->sphi || !m->rho || !m->Y) {
    nbp_destroy(m);
    return NBO_EINVAL;
  }
  /* azimuthal bins: midpoints phi_p = 2 pi (p + 1/2) / n_phi */
  for (int64_t q = 0; q < m->NP; ++q) {
    const double ph = 2.0 * P_PI * (q + 0.5) / m->NP;
    m->cphi[q] = m->ext ? cos(ph) : 0.0;
    m->sphi[q] = m->ext ? sin(ph) : 0.0;
  }
  /* number luminosities N = L / <E>, <E> = T F3 / F2; index 3 is anti-nu_x */
  double T[4], L[4];
  for (int a = 0; a < 3; ++a) { T[a] = p->temp_mev[a]; L[a] = p->lum_erg_s[a]; }
  T[3] = (p->temp_xbar_mev != 0.0) ? p->temp_xbar_mev : p->temp_mev[2];
  L[3] = (p->temp_xbar_mev != 0.0) ? p->lum_xbar_erg_s : p->lum_erg_s[2];
  double N[4];
  for (int a = 0; a < 4; ++a) N[a] = L[a] * P_ERG_MEV / (T[a] * P_F3 / P_F2);
  const double pref = kappa0 * m->du * m->dE / m->NP;
  /* 3f mixing matrix U = R23 U13 R12 (delta = 0) */
  double U[3][3] = {{0}};
  if (m->n == 3) {
    const double c12 = cos(p->theta[0]), s12 = sin(p->theta[0]);
    const double c13 = cos(p->theta[1]), s13 = sin(p->theta[1]);
    const double c23 = cos(p->theta[2]), s23 = sin(p->theta[2]);
    const double R23[3][3] = {{1, 0, 0}, {0, c23, s23}, {0, -s23, c23}};
    const double U13[3][3] = {{c13, 0, s13}, {0, 1, 0}, {-s13, 0, c13}};
    const double R12[3][3] = {{c12, s12, 0}, {-s12, c12, 0}, {0, 0, 1}};
    double A[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        A[i][j] = 0.0;
        for (int l = 0; l < 3; ++l) A[i][j] += U13[i][l] * R12[l][j];
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) U[i][j] += R23[i][l] * A[l][j];
  }
  for (int64_t k = 0; k < m->NE; ++k) {
    const double E = p->e_min_mev + (k + 0.5) * m->dE;
    m->E[k] = E;
    const double f[4] = {fermi_dirac(E, T[0]), fermi_dirac(E, T[1]), fermi_dirac(E, T[2]),
                         fermi_dirac(E, T[3])};
    for (int s = 0; s < m->ns; ++s) {
      double w;
      if (!p->species4)   /* heavy-flavour-born states = I - rho_e (unitarity) */
        w = m->anti[s] ? N[1] * f[1] - N[3] * f[3] : N[0] * f[0] - N[2] * f[2];
      else if (m->flav[s] == 0)
        w = m->anti[s] ? N[1] * f[1] : N[0] * f[0];
      else
        w = m->anti[s] ? N[3] * f[3] : N[2] * f[2];
      m->g[s * m->NE + k] = pref * w;
    }
    mat H = m_zero();
    if (m->n == 2) {
      /* dm^2 / 4E in km^-1 (E in MeV) */
      const double om = p->dm2_ev2[0] / (4.0 * E * 1.0e6) / P_HBARC_EV_KM;
      const double c2 = cos(2.0 * p->theta[0]), s2 = sin(2.0 * p->theta[0]);
      H.a[0][0] = -om * c2; H.a[0][1] = om * s2;
      H.a[1][0] = om * s2;  H.a[1][1] = om * c2;
    } else {
      const double m2[3] = {0.0, p->dm2_ev2[0], p->dm2_ev2[1]};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int l = 0; l < 3; ++l) v += U[i][l] * m2[l] * U[j][l];
          H.a[i][j] = v / (2.0 * E * 1.0e6) / P_HBARC_EV_KM;
        }
    }
    m->hvac[k] = H;
  }
  nbp_reset(m);
  *out = m;
  return NBO_OK;
}

void nbp_destroy(plain_model *m) {
  if (!m) return;
  free(m->E); free(m->g); free(m->hvac); free(m->cphi); free(m->sphi); free(m->rho); free(m->Y);
  free(m);
}

int64_t nbp_n_beams(const plain_model *m) { return m->nb; }
int64_t nbp_step_index(const plain_model *m) { return m->step; }

/* every beam in the flavour eigenstate of its birth (Sec. 3.4) */
int nbp_reset(plain_model *m) {
  for (int64_t b = 0; b < m->nb; ++b) {
    int s;
    int64_t j, q, k;
    beam_of(m, b, &s, &j, &q, &k);
    m->rho[b] = m_zero();
    m->rho[b].a[m->flav[s]][m->flav[s]] = 1.0;
  }
  m->step = 0;
  return NBO_OK;
}

/* The moments of the states S at radius r (Eqs. Hnu, F): per (species, emission[,
 * azimuth]) row the energy sum first, then the rows in order. */
static void moments(const plain_model *m, const mat *S, double r, moments_t *out) {
  const int n = m->n;
  const int64_t nrow = (int64_t)m->ns * m->NU * m->NP;
  moments_t *part = (moments_t *)calloc((size_t)nrow, sizeof(moments_t));
#pragma omp parallel for schedule(static)
  for (int64_t row = 0; row < nrow; ++row) {
    const int s = (int)(row / (m->NU * m->NP));
    const int64_t j = (row / m->NP) % m->NU, q = row % m->NP;
    mat E = m_zero();   /* sum_k g rho~ */
    for (int64_t k = 0; k < m->NE; ++k) {
      const mat *x = S + row * m->NE + k;
      const double w = m->g[s * m->NE + k];
      for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c)
          E.a[a][c] += w * (m->anti[s] ? -conj(x->a[a][c]) : x->a[a][c]);
    }
    const double ct = cos_theta(m, j, r);
    const double st = m->ext ? sin_theta(m, j, r) : 0.0;
    moments_t *t = part + row;
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) {
        t->J[0].a[a][c] = E.a[a][c] / ct;
        t->J[1].a[a][c] = E.a[a][c];
        t->J[2].a[a][c] = E.a[a][c] * (st * m->cphi[q] / ct);
        t->J[3].a[a][c] = E.a[a][c] * (st * m->sphi[q] / ct);
      }
  }
  memset(out, 0, sizeof *out);
  for (int64_t row = 0; row < nrow; ++row)
    for (int i = 0; i < 4; ++i)
      for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c) out->J[i].a[a][c] += part[row].J[i].a[a][c];
  free(part);
}

/* H of beam b at radius r for the moments J (Eq. eom with Eq. Hnu) */
static mat hamiltonian(const plain_model *m, int64_t b, double r, const moments_t *J) {
  int s;
  int64_t j, q, k;
  beam_of(m, b, &s, &j, &q, &k);
  const int n = m->n;
  const double ct = cos_theta(m, j, r);
  const double st = m->ext ? sin_theta(m, j, r) : 0.0;
  const double mu = 0.5 * (m->R / r) * (m->R / r);
  double qp = 1.0;
  for (int i = 0; i < m->p.ne_power; ++i) qp *= m->R / r;
  const double lam = m->lam0 * qp;
  mat H = m->hvac[k];
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < n; ++c) {
      zc nn = J->J[0].a[a][c] - ct * J->J[1].a[a][c];
      if (m->ext) nn -= st * (m->cphi[q] * J->J[2].a[a][c] + m->sphi[q] * J->J[3].a[a][c]);
      nn *= mu;
      if (m->anti[s]) H.a[a][c] -= conj(nn);
      else H.a[a][c] += nn;
    }
  H.a[0][0] += m->anti[s] ? -lam : lam;
  return H;
}

/* stage generator F = -i (h / c_b(r)) H_b(r, J) */
static mat generator(const plain_model *m, int64_t b, double r, double h, const moments_t *J) {
  int s;
  int64_t j, q, k;
  beam_of(m, b, &s, &j, &q, &k);
  const mat H = hamiltonian(m, b, r, J);
  const double a = h / cos_theta(m, j, r);
  return m_lin(m->n, -I * a, &H, 0.0, &H);
}

/* one fixed step of the Lie-group RK4 (see the header) */
static void step_once(plain_model *m) {
  const int n = m->n;
  const double h = m->h;
  const double r0 = m->p.r_start_km + m->step * h;
  const double rm = r0 + 0.5 * h;
  const double r1 = m->p.r_start_km + (m->step + 1) * h;
  moments_t J1, J2, J3, J4;
  moments(m, m->rho, r0, &J1);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nb; ++b) {
    const mat F1 = generator(m, b, r0, h, &J1);
    const mat Om = m_lin(n, 0.5, &F1, 0.0, &F1);
    m->Y[b] = conjugate(n, &Om, &m->rho[b]);
  }
  moments(m, m->Y, rm, &J2);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nb; ++b) {
    const mat F1 = generator(m, b, r0, h, &J1);
    const mat F2 = generator(m, b, rm, h, &J2);
    const mat C = m_comm(n, &F1, &F2);
    const mat Om = m_lin(n, 0.5, &F2, -0.125, &C);
    m->Y[b] = conjugate(n, &Om, &m->rho[b]);
  }
  moments(m, m->Y, rm, &J3);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nb; ++b) {
    const mat F3 = generator(m, b, rm, h, &J3);
    m->Y[b] = conjugate(n, &F3, &m->rho[b]);
  }
  moments(m, m->Y, r1, &J4);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nb; ++b) {
    const mat F1 = generator(m, b, r0, h, &J1);
    const mat F2 = generator(m, b, rm, h, &J2);
    const mat F3 = generator(m, b, rm, h, &J3);
    const mat F4 = generator(m, b, r1, h, &J4);
    mat S = m_lin(n, 1.0, &F1, 2.0, &F2);
    S = m_lin(n, 1.0, &S, 2.0, &F3);
    S = m_lin(n, 1.0, &S, 1.0, &F4);
    const mat C = m_comm(n, &F1, &F4);
    const mat Th = m_lin(n, 1.0 / 6.0, &S, -1.0 / 12.0, &C);
    mat x = conjugate(n, &Th, &m->rho[b]);
    if (m->p.renorm) renormalise(n, &x);
    m->rho[b] = x;
  }
  m->step += 1;
}

int nbp_step(plain_model *m, int64_t steps) {
  if (!m || steps < 0) return NBO_EINVAL;
  for (int64_t i = 0; i < steps && m->step < m->p.n_steps; ++i) {
    step_once(m);
    /* a non-finite state is a numerical failure */
    for (int64_t b = 0; b < m->nb; ++b)
      if (!isfinite(creal(m->rho[b].a[0][0]))) return NBO_ENUMERIC;
  }
  return NBO_OK;
}

/* Re rho_ee of every beam (the survival probability; rhobar_ee for antineutrinos) */
int nbp_read_pee(const plain_model *m, double *out) {
  for (int64_t b = 0; b < m->nb; ++b) out[b] = creal(m->rho[b].a[0][0]);
  return NBO_OK;
}

/* rho of every beam as [nb][n][n] complex (interleaved re, im) */
int nbp_get_rho(const plain_model *m, double *out) {
  const int n = m->n;
  for (int64_t b = 0; b < m->nb; ++b)
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) {
        out[((b * n + a) * n + c) * 2] = creal(m->rho[b].a[a][c]);
        out[((b * n + a) * n + c) * 2 + 1] = cimag(m->rho[b].a[a][c]);
      }
  return NBO_OK;
}
int nbp_set_rho(plain_model *m, const double *in, int64_t step) {
  const int n = m->n;
  for (int64_t b = 0; b < m->nb; ++b) {
    m->rho[b] = m_zero();
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c)
        m->rho[b].a[a][c] = in[((b * n + a) * n + c) * 2] + I * in[((b * n + a) * n + c) * 2 + 1];
  }
  m->step = step;
  return NBO_OK;
}

/* Moments of the current state at radius r as [4][n][n] complex (J0, J1, Jsc, Jss). */
int nbp_moments(const plain_model *m, double r, double *out) {
  moments_t J;
  moments(m, m->rho, r, &J);
  const int n = m->n;
  for (int i = 0; i < 4; ++i)
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) {
        out[((i * n + a) * n + c) * 2] = creal(J.J[i].a[a][c]);
        out[((i * n + a) * n + c) * 2 + 1] = cimag(J.J[i].a[a][c]);
      }
  return NBO_OK;
}
/* H of every beam at radius r for the moments of the current state, [nb][n][n] complex */
int nbp_hamiltonian(const plain_model *m, double r, double *out) {
  moments_t J;
  moments(m, m->rho, r, &J);
  const int n = m->n;
  for (int64_t b = 0; b < m->nb; ++b) {
    const mat H = hamiltonian(m, b, r, &J);
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) {
        out[((b * n + a) * n + c) * 2] = creal(H.a[a][c]);
        out[((b * n + a) * n + c) * 2 + 1] = cimag(H.a[a][c]);
      }
  }
  return NBO_OK;
}
/* exp(-i K) of a Hermitian n x n matrix (interleaved complex), for the pins */
void nbp_expm(int n, const double *k, double *out) {
  mat Om = m_zero();
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < n; ++c)
      Om.a[a][c] = -I * (k[(a * n + c) * 2] + I * k[(a * n + c) * 2 + 1]);
  const mat E = expm_antiherm(n, &Om);
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < n; ++c) {
      out[(a * n + c) * 2] = creal(E.a[a][c]);
      out[(a * n + c) * 2 + 1] = cimag(E.a[a][c]);
    }
}
