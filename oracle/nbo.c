/*
 * nbo.c -- CPU oracle for the bulb-model radial stepper: plain, slow FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY (see nbo.h).  Nothing in the product path links this file.
 *
 * What is computed, and where the paper defines it:
 *   - bins equal in E and in u = sin^2(theta_R)                    (Sec. 3.2)
 *   - H_vac (2f form in Sec. 2; 3f = U diag(0,dm21,dm31) U^+/2E),
 *     H_mat = sqrt2 G_F n_e diag(1,0[,0])                          (Sec. 2)
 *   - H_nunu from the beam sum of Eq. Hnu with the weights of F;
 *     the cos(theta') integral at radius r is done over the emission variable u,
 *     d cos(theta') = (R^2/2r^2) du / cos(theta'), which factors H_nunu into two
 *     moments J0 = sum g rho~/c and J1 = sum g rho~                (Eqs. Hnu, F)
 *   - antineutrinos evolve with H_vac - H_mat - H_nunu^*           (Eq. eom)
 *   - initial states: flavour eigenstates at the start radius      (Sec. 3.4)
 *   - one-step propagator exp(-i H dl), dl = dr / cos(theta)       (Eq. U)
 *     used as the exponential map of a Lie-group RK4 (Munthe-Kaas 1999):
 *       F_i = -i (h/c) H(r_i, Y_i),  Y_1 = rho_n,
 *       Y_2 = e^{F_1/2} rho_n e^{-F_1/2},
 *       Y_3 = e^{F_2/2 - [F_1,F_2]/8} ...,  Y_4 = e^{F_3} ...,
 *       rho_{n+1} = e^{Theta} rho_n e^{-Theta},
 *       Theta = (F_1 + 2F_2 + 2F_3 + F_4)/6 - [F_1,F_4]/12.
 *     Two flavours: rho = (1 + P.sigma)/2 and e^{F} rotates P about (h/c)B by |(h/c)B|,
 *     with H = B.sigma/2 + trace (so [X,Y] maps to the cross product).
 *     Three flavours: the state is the wavefunction psi of Eq. psi (rho = psi psi^+);
 *     e^{-iK} psi is evaluated exactly (isolated eigenvector + the 2x2 propagator of
 *     Eq. U on the orthogonal plane).
 *
 * Pins (tests/test_oracle_pins.py): units against hand values, spectra against
 * quadrature, sin/cos against libm, rotations and exp(-iK) against SciPy, the fixed-point
 * sum against exact rationals, vacuum and constant-density MSW closed forms (2f and 3f),
 * the factored H_nunu against the direct beam-pair sum of Eq. Hnu, norm conservation,
 * the flux-weighted polarisation invariant, single-angle = one angle bin, two tracked
 * species = every flavour explicit, 4th-order convergence, plain RK4 agreement.
 * Adjoint pins (tests/test_oracle_adjoint.py): central differences of the forward
 * integration for all five parameters and for the initial state, the closed-form vacuum
 * derivative in theta_v, linearity in the cotangent, checkpoint-period independence.
 * The full nonlinear bulb evolution at benchmark scale has no external reference (the
 * paper's result is a figure without data): parity unpinned beyond its parts.
 *
 * Arithmetic specification.  The GPU library implements the same operation order
 * from its own sources, so that results agree bit for bit on any input:
 *   - no contraction (built with -ffp-contract=off); fma() only where written;
 *   - sin/cos: own Cody-Waite reduction + Taylor polynomials (sincos_spec);
 *   - moment sums are exact fixed-point integer sums, independent of order.
 */
#include "nbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

/* ---------------------------------------------------------------- constants */
/* sqrt(2) G_F (hbar c)^3 expressed in km^-1 cm^3 (G_F = 1.1663787e-5 GeV^-2,
 * hbar c = 1.973269804e-14 GeV cm = 1.973269804e-19 GeV km). */
static double sqrt2gf_km_cm3(void) {
  const double hc_cm = 1.973269804e-14, hc_km = 1.973269804e-19;
  return (1.4142135623730951 * 1.1663787e-5) * ((hc_cm * hc_cm) * hc_cm) / hc_km;
}
#define VAC_K (1.0 / (4.0e6 * 1.973269804e-10)) /* dm^2[eV^2]/(4E[MeV]) -> km^-1 */
#define ERG_MEV 624150.9074460763
#define C_CM_S 2.99792458e10
#define PI_D 3.141592653589793
#define F2_0 1.8030853547393914  /* int x^2/(e^x+1) = 3 zeta(3)/2 */
#define F3_0 5.682196976983475   /* int x^3/(e^x+1) = 7 pi^4/120 */
#define TWO62 4611686018427387904.0
#define TWO64 18446744073709551616.0

/* --------------------------------------------------------------- sin / cos */
/* Cody-Waite reduction by pi/2 (three-part split, fma), Taylor polynomials of
 * degree 17 (sin) and 18 (cos) on |r| <= pi/4.  The multiple k is the exact product
 * x 2/pi rounded once to the nearest integer: fma adds 1.5 2^52 and rounds in a binade of
 * unit spacing, so t - 1.5 2^52 = k and the low bits of t are k mod 4 (|x| < 2^50). */
static const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
static const double PIO2_HI = 0x1.921fb54442d18p+0;
static const double PIO2_MID = 0x1.1a62633145c07p-54;
static const double PIO2_LO = -0x1.f1976b7ed8fbcp-110;

static void sincos_spec(double x, double *sn, double *cs) {
  const double t = fma(x, TWO_OVER_PI, 0x1.8p52);
  const double k = t - 0x1.8p52;
  double r = fma(-k, PIO2_HI, x);
  r = fma(-k, PIO2_MID, r);
  r = fma(-k, PIO2_LO, r);
  const double r2 = r * r;
  double ps = 1.0 / 355687428096000.0;
  ps = fma(ps, r2, -1.0 / 1307674368000.0);
  ps = fma(ps, r2, 1.0 / 6227020800.0);
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double s = fma(r2 * r, ps, r);
  double pc = -1.0 / 6402373705728000.0;
  pc = fma(pc, r2, 1.0 / 20922789888000.0);
  pc = fma(pc, r2, -1.0 / 87178291200.0);
  pc = fma(pc, r2, 1.0 / 479001600.0);
  pc = fma(pc, r2, -1.0 / 3628800.0);
  pc = fma(pc, r2, 1.0 / 40320.0);
  pc = fma(pc, r2, -1.0 / 720.0);
  pc = fma(pc, r2, 1.0 / 24.0);
  pc = fma(pc, r2, -0.5);
  const double c = fma(r2, pc, 1.0);
  uint64_t tb;
  memcpy(&tb, &t, sizeof tb);
  switch ((int)(tb & 3)) {
    case 0: *sn = s; *cs = c; break;
    case 1: *sn = c; *cs = -s; break;
    case 2: *sn = -s; *cs = -c; break;
    default: *sn = -c; *cs = s; break;
  }
}

/* ------------------------------------------------------------- fixed point */
/* One per-angle term v of J0 becomes the integer trunc(v 2^e); |v 2^e| < limit = 2^62 is
 * required. */
static inline int64_t to_fix(double v, double scale, double limit, int *err) {
  const double x = v * scale;
  if (!(fabs(x) < limit)) { *err = 1; return 0; }
  return (int64_t)x;
}
/* A beam's moment contribution: the exact product v ws (ws = w 2^e1, the weight in units
 * of the fixed-point step) rounded once to the nearest integer, ties to even.  fma adds
 * 1.5 2^52 to the exact product and rounds in a binade of unit spacing, so the integer
 * sits in the low mantissa bits; this is exact for |v ws| <= 2^51, which the state check
 * of the caller (squared norm below 2, so |v| < 2, and |ws| < 2^50 by the choice of e1)
 * guarantees. */
static inline int64_t fix_round(double v, double ws) {
  const double t = fma(v, ws, 0x1.8p52);
  int64_t b;
  memcpy(&b, &t, sizeof b);
  return b - (int64_t)0x4338000000000000LL;
}
/* Integer -> double in sign-magnitude form: |x| = hi 2^64 + lo, each half converted
 * (round to nearest) and added; the sign is applied last. */
static inline double i128_to_double(i128 x) {
  const int neg = x < 0;
  const unsigned __int128 a = neg ? (unsigned __int128)(-x) : (unsigned __int128)x;
  const uint64_t hi = (uint64_t)(a >> 64), lo = (uint64_t)a;
  const double v = (double)hi * TWO64 + (double)lo;
  return neg ? -v : v;
}

/* ---------------------------------------------------------- complex helpers */
typedef struct { double re, im; } cx;
static inline cx cx_make(double re, double im) { cx r; r.re = re; r.im = im; return r; }
static inline cx cx_mul(cx a, cx b) {
  return cx_make(fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re));
}
static inline cx cx_mulc(cx a, cx b) { /* a * conj(b) */
  return cx_make(fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -(a.re * b.im)));
}
static inline cx cx_cjmul(cx a, cx b) { /* conj(a) * b */
  return cx_make(fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re)));
}
static inline cx cx_rmul(double a, cx b) { return cx_make(a * b.re, a * b.im); }
static inline cx cx_add(cx a, cx b) { return cx_make(a.re + b.re, a.im + b.im); }
static inline cx cx_sub(cx a, cx b) { return cx_make(a.re - b.re, a.im - b.im); }
static inline cx cx_conj(cx a) { return cx_make(a.re, -a.im); }
static inline double cx_norm2(cx a) { return fma(a.re, a.re, a.im * a.im); }

/* Hermitian 3x3: real diagonal d[0..2], upper off-diagonals o[0]=(0,1), o[1]=(0,2), o[2]=(1,2). */
typedef struct { double d[3]; cx o[3]; } herm3;
static inline cx h3_at(const herm3 *h, int a, int b) {
  if (a == b) return cx_make(h->d[a], 0.0);
  if (a < b) return h->o[a + b - 1];
  return cx_conj(h->o[a + b - 1]);
}

/* a0 b0 + a1 b1 + a2 b2 (complex), the six real products accumulated with fma from the
 * last one up: the fused form of every three-term complex dot product below. */
static inline cx dot3_mul(cx a0, cx b0, cx a1, cx b1, cx a2, cx b2) {
  return cx_make(fma(a0.re, b0.re, fma(-a0.im, b0.im, fma(a1.re, b1.re, fma(-a1.im, b1.im,
                     fma(a2.re, b2.re, -(a2.im * b2.im)))))),
                 fma(a0.re, b0.im, fma(a0.im, b0.re, fma(a1.re, b1.im, fma(a1.im, b1.re,
                     fma(a2.re, b2.im, a2.im * b2.re))))));
}

/* C(A,B) = i [A,B] (Hermitian for Hermitian A, B). */
static herm3 h3_icomm(const herm3 *A, const herm3 *B) {
  cx X[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      X[a][b] = dot3_mul(h3_at(A, a, 0), h3_at(B, 0, b), h3_at(A, a, 1), h3_at(B, 1, b),
                         h3_at(A, a, 2), h3_at(B, 2, b));
  herm3 C;
  for (int a = 0; a < 3; ++a) C.d[a] = -2.0 * X[a][a].im;
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int t = 0; t < 3; ++t) {
    const cx xab = X[pa[t]][pb[t]], xba = X[pb[t]][pa[t]];
    const double dre = xab.re - xba.re, dim = xab.im + xba.im;
    C.o[t] = cx_make(-dim, dre);
  }
  return C;
}

/* u^+ v */
static inline cx inner3(const cx u[3], const cx v[3]) {
  return dot3_mul(cx_conj(u[0]), v[0], cx_conj(u[1]), v[1], cx_conj(u[2]), v[2]);
}
/* |v0|^2 + |v1|^2 + |v2|^2 */
static inline double norm3(const cx v[3]) {
  return fma(v[0].re, v[0].re, fma(v[0].im, v[0].im, fma(v[1].re, v[1].re, fma(v[1].im, v[1].im,
             fma(v[2].re, v[2].re, v[2].im * v[2].im)))));
}

/* psi' = exp(-i K) psi up to a global phase, for Hermitian K.
 * With K0 the traceless part, l1 its eigenvalue of largest magnitude (simple and well
 * separated from the other two), v1 its eigenvector and P the projector on the plane
 * orthogonal to v1: on that plane K0 - hm (hm = -l1/2, the mean of the other two
 * eigenvalues) squares to th^2 times the identity, so
 *   exp(-i K0) psi = e^{-i l1} (v1^+ psi) v1
 *                  + e^{-i hm} [cos(th) P psi - i sin(th)/th (K0 - hm) P psi],
 * the 2x2 propagator of Eq. U on the plane, th = |(K0 - hm) w| / |w| for any w in the
 * plane (here w = P psi).  The traces (of K, and e^{-i hm}) only contribute global phases.
 * v1 is kept unnormalised (v1 = c / |c| with c a column of adj(K0 - l1)), so intermediate
 * magnitudes grow like |K0|^5; with the sin/cos reduction (phases below 2^50) the form
 * holds for 2^-100 < |K0| < 1e15, and |K0|^2 / 2 <= 2^-200 is taken as K0 = 0 (error below
 * 1e-30). */
static void exp3_apply(const herm3 *K, const cx psi[3], cx out[3]) {
  const double tr = ((K->d[0] + K->d[1]) + K->d[2]) * (1.0 / 3.0);
  const double a0 = K->d[0] - tr, a1 = K->d[1] - tr, a2 = K->d[2] - tr;
  const cx x = K->o[0], y = K->o[1], z = K->o[2];
  const double nx = cx_norm2(x), ny = cx_norm2(y), nz = cx_norm2(z);
  const double s2 = fma(a0, a0, fma(a1, a1, a2 * a2));
  const double p = fma(0.5, s2, (nx + ny) + nz);               /* Tr K0^2 / 2 */
  const cx xz = cx_mul(x, z);
  const double t = fma(xz.re, y.re, xz.im * y.im);             /* Re(x z conj(y)) */
  const double q = fma(a0, fma(a1, a2, -nz), fma(-a1, ny, fma(-a2, nx, 2.0 * t))); /* det */
  if (!(p > 0x1p-200)) { out[0] = psi[0]; out[1] = psi[1]; out[2] = psi[2]; return; }
  /* largest-magnitude root of l^3 - p l - q: 3 Halley steps l - f f' / (f'^2 - f f''/2)
   * (f'' = 6 l) on the |q| problem.  The root's magnitude lies in [sqrt(p), 2 sqrt(p/3)];
   * the start is 2 sqrt(p/3) by halving the exponent in the bit pattern of p/3 (the
   * mantissa interpolated linearly: at most 6.1 % above the square root, never below), so
   * it is above the root and within 23 % of it, and three cubic steps reach full FP64
   * accuracy (worst 1.63e-16 over 2e6 spectra of every shape and scale) */
  const double sg = (q < 0.0) ? -1.0 : 1.0;
  const double qa = sg * q;
  double lam;
  {
    const double x = p * (1.0 / 3.0);
    uint64_t i;
    memcpy(&i, &x, sizeof i);
    i = (i >> 1) + 0x1FF8000000000000ULL;
    memcpy(&lam, &i, sizeof lam);
    lam = 2.0 * lam;
  }
  for (int it = 0; it < 3; ++it) {
    const double l2 = lam * lam;
    const double fv = fma(lam, l2 - p, -qa);
    const double dv = fma(3.0, l2, -p);
    const double den = fma(dv, dv, -((3.0 * lam) * fv));
    lam = lam - (fv * dv) / den;
  }
  const double l1 = sg * lam;
  /* eigenvector: a column of adj(K0 - l1 I), which has rank one (mu v1 v1^+ with
   * mu = (l2 - l1)(l3 - l1) > 0), the one with the largest diagonal entry (first wins
   * ties; the largest |v1_j|, so the best-conditioned column).  With p_i = a_i - l1 the
   * cofactors are c00 = p1 p2 - |z|^2, c11 = p0 p2 - |y|^2, c22 = p0 p1 - |x|^2 and the
   * entries above the diagonal u = y z^* - p2 x, v = x z - p1 y, t = x^* y - p0 z, so the
   * columns are (c00, u^*, v^*), (u, c11, t^*) and (v, t, c22). */
  const double p0 = a0 - l1, p1 = a1 - l1, p2 = a2 - l1;
  const double c00 = fma(p1, p2, -nz), c11 = fma(p0, p2, -ny), c22 = fma(p0, p1, -nx);
  const cx u = cx_make(fma(y.re, z.re, fma(y.im, z.im, -(p2 * x.re))),
                       fma(y.im, z.re, fma(-y.re, z.im, -(p2 * x.im))));
  const cx v = cx_make(fma(x.re, z.re, fma(-x.im, z.im, -(p1 * y.re))),
                       fma(x.re, z.im, fma(x.im, z.re, -(p1 * y.im))));
  const cx tt = cx_make(fma(x.re, y.re, fma(x.im, y.im, -(p0 * z.re))),
                        fma(x.re, y.im, fma(-x.im, y.re, -(p0 * z.im))));
  int jc = 0;
  double cjj = c00;
  if (c11 > cjj) { jc = 1; cjj = c11; }
  if (c22 > cjj) { jc = 2; cjj = c22; }
  cx best[3];
  if (jc == 0) { best[0] = cx_make(c00, 0.0); best[1] = cx_conj(u); best[2] = cx_conj(v); }
  else if (jc == 1) { best[0] = u; best[1] = cx_make(c11, 0.0); best[2] = cx_conj(tt); }
  else { best[0] = v; best[1] = tt; best[2] = cx_make(c22, 0.0); }
  const double nb = norm3(best);
  if (!(nb > 0.0)) { out[0] = psi[0]; out[1] = psi[1]; out[2] = psi[2]; return; }
  const double hm = -0.5 * l1;
  const double d0 = a0 - hm, d1 = a1 - hm, d2 = a2 - hm;
  /* (K0 - hm) v for a vector v: rows (d0, x, y), (x^*, d1, z), (y^*, z^*, d2), each a
   * complex dot product with the real diagonal entry, fused from the last product up */
#define NB_KMV(v, o)                                                                          \
  do {                                                                                      \
    (o)[0] = cx_make(fma(d0, (v)[0].re, fma(x.re, (v)[1].re, fma(-x.im, (v)[1].im,          \
                         fma(y.re, (v)[2].re, -(y.im * (v)[2].im))))),                      \
                     fma(d0, (v)[0].im, fma(x.re, (v)[1].im, fma(x.im, (v)[1].re,           \
                         fma(y.re, (v)[2].im, y.im * (v)[2].re)))));                        \
    (o)[1] = cx_make(fma(x.re, (v)[0].re, fma(x.im, (v)[0].im, fma(d1, (v)[1].re,           \
                         fma(z.re, (v)[2].re, -(z.im * (v)[2].im))))),                      \
                     fma(x.re, (v)[0].im, fma(-x.im, (v)[0].re, fma(d1, (v)[1].im,          \
                         fma(z.re, (v)[2].im, z.im * (v)[2].re)))));                        \
    (o)[2] = cx_make(fma(y.re, (v)[0].re, fma(y.im, (v)[0].im, fma(z.re, (v)[1].re,         \
                         fma(z.im, (v)[1].im, d2 * (v)[2].re)))),                           \
                     fma(y.re, (v)[0].im, fma(-y.im, (v)[0].re, fma(z.re, (v)[1].im,        \
                         fma(-z.im, (v)[1].re, d2 * (v)[2].im)))));                         \
  } while (0)
  /* al = (c^+ psi) / |c|^2, so that (v1^+ psi) v1 = al c */
  const cx al = cx_rmul(1.0 / nb, inner3(best, psi));
  cx pp[3], kp[3];
  /* P psi = psi - al c */
  for (int c = 0; c < 3; ++c)
    pp[c] = cx_make(fma(-al.re, best[c].re, fma(al.im, best[c].im, psi[c].re)),
                    fma(-al.re, best[c].im, fma(-al.im, best[c].re, psi[c].im)));
  NB_KMV(pp, kp);
#undef NB_KMV
  /* (K0 - hm)^2 = th^2 on the plane: th = |(K0 - hm) P psi| / |P psi|, 0 for P psi = 0 (a
   * rounding-level component of P psi along v1 perturbs th only where P psi itself is of
   * that order, so the result stays within rounding of the exact one) */
  const double npp = norm3(pp);
  const double th = (npp > 0.0) ? sqrt(norm3(kp) / npp) : 0.0;
  const double phi = l1 - hm;
  double sp, cp, st, ct;
  sincos_spec(phi, &sp, &cp);
  sincos_spec(th, &st, &ct);
  const double sc = (th > 0.0) ? st / th : 1.0;
  const cx ap = cx_mul(al, cx_make(cp, -sp));
  /* ap c + cos(th) P psi - i sin(th)/th (K0 - hm) P psi */
  for (int c = 0; c < 3; ++c)
    out[c] = cx_make(fma(ap.re, best[c].re, fma(-ap.im, best[c].im, fma(ct, pp[c].re, sc * kp[c].im))),
                     fma(ap.re, best[c].im, fma(ap.im, best[c].re, fma(ct, pp[c].im, -(sc * kp[c].re)))));
}

/* Rotation of the Bloch vector P about x by the angle |x| (2x2 form of Eq. U as a
 * unit quaternion (cos|x|/2, sin(|x|/2) x/|x|)). */
static void rotate2(const double x[3], const double P[3], double out[3]) {
  const double t2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
  const double th = sqrt(t2);
  if (th == 0.0) { out[0] = P[0]; out[1] = P[1]; out[2] = P[2]; return; }
  double s, c;
  sincos_spec(0.5 * th, &s, &c);
  const double k = s / th;
  const double v0 = x[0] * k, v1 = x[1] * k, v2 = x[2] * k;
  double t0 = v1 * P[2] - v2 * P[1];
  double t1 = v2 * P[0] - v0 * P[2];
  double tt = v0 * P[1] - v1 * P[0];
  t0 = t0 + t0; t1 = t1 + t1; tt = tt + tt;
  const double u0 = v1 * tt - v2 * t1;
  const double u1 = v2 * t0 - v0 * tt;
  const double u2 = v0 * t1 - v1 * t0;
  out[0] = (P[0] + c * t0) + u0;
  out[1] = (P[1] + c * t1) + u1;
  out[2] = (P[2] + c * tt) + u2;
}

/* ------------------------------------------------------------------- model */
struct nbo_model {
  nbo_params p;
  int nf, ncomp, nsc;       /* flavours, moment components, state components */
  int ns;                   /* species rows */
  int anti[6], init_flav[6];
  int64_t NE, NU, NP, nb;   /* energy, emission and azimuthal bins (NP = 1: bulb) */
  int ext;                  /* extended bulb model (n_phi >= 1) */
  double *cphi, *sphi;      /* cos and sin of the azimuth of every azimuthal bin */
  double dE, du, h, R, lam0, kappa0;
  double *E, *w;            /* E[k]; w[s*NE + k] (includes kappa0 du dE) */
  double *bv;               /* 2f: bx,bz per k; 3f: 6 per k (d0,d1,d2,o01,o02,o12) */
  double v0[6];             /* 3f: the vacuum Hamiltonian times E (bv of bin k = v0 / E_k) */
  double *ek;               /* 3f: e_k = 1 / E_k */
  double s1, s0, p2e1, p2e0;/* fixed-point scales 2^e1, 2^e0 and their inverses */
  int e1, e0;
  double *X;                /* state [nb][nsc] */
  double *Y;                /* stage scratch [nb][nsc] */
  int64_t step;
};

typedef struct { double r, q, q2, lam, mu; } radial;

static radial radial_at(const nbo_model *m, double r) {
  radial g;
  g.r = r;
  g.q = m->R / r;
  g.q2 = g.q * g.q;
  double qp = 1.0;
  for (int i = 0; i < m->p.ne_power; ++i) qp = qp * g.q;
  g.lam = m->lam0 * qp;     /* sqrt2 G_F n_e(r) */
  g.mu = 0.5 * g.q2;        /* R^2/(2 r^2): Jacobian of d cos(theta') -> du */
  return g;
}
static inline double u_of(const nbo_model *m, int64_t j) { return ((double)j + 0.5) / (double)m->NU; }
static inline double c_of(const radial *g, double u) { return sqrt(1.0 - u * g->q2); }
/* sin(theta) at radius r of emission bin u: sin(theta) r = sin(theta_R) R */
static inline double s_of(const radial *g, double u) { return sqrt(u * g->q2); }

/* Beam b = ((s n_u + j) n_phi + p) n_energy + k -> its species, emission, azimuthal and
 * energy bins. */
static inline void beam_of(const nbo_model *m, int64_t b, int *s, int64_t *j, int64_t *p, int64_t *k) {
  *k = b % m->NE;
  const int64_t row = b / m->NE;
  *p = row % m->NP;
  *j = (row / m->NP) % m->NU;
  *s = (int)(row / (m->NP * m->NU));
}
/* Geometry of a beam at one radius: cos(theta), sin(theta), cos(phi), sin(phi). */
typedef struct { double c, sn, cp, sp; } bgeo;
static bgeo geo_of(const nbo_model *m, const radial *g, int64_t j, int64_t p) {
  bgeo o;
  const double u = u_of(m, j);
  o.c = c_of(g, u);
  o.sn = m->ext ? s_of(g, u) : 0.0;
  o.cp = m->ext ? m->cphi[p] : 0.0;
  o.sp = m->ext ? m->sphi[p] : 0.0;
  return o;
}

static double fermi_dirac(double E, double T) {
  return (E * E) / ((F2_0 * ((T * T) * T)) * (exp(E / T) + 1.0));
}

int nbo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#endif
  return n;
}

int nbo_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int nbo_create(const nbo_params *p, nbo_model **out) {
  *out = NULL;
  if (!p || (p->n_flavor != 2 && p->n_flavor != 3) || p->n_energy < 1 || p->n_u < 1 ||
      p->n_steps < 1 || !(p->r_start_km >= p->r_nu_km) || !(p->r_end_km > p->r_start_km) ||
      !(p->e_max_mev > p->e_min_mev) || !(p->e_min_mev > 0.0) || p->delta_cp != 0.0 ||
      p->ne_power < 0 || p->ne_power > 8 || !(p->r_nu_km > 0.0) || p->n_phi < 0 ||
      p->n_phi > 4096)
    return NBO_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!(p->temp_mev[i] > 0.0) || !(p->lum_erg_s[i] >= 0.0)) return NBO_EINVAL;
  if (p->temp_xbar_mev != 0.0 && (!(p->temp_xbar_mev > 0.0) || !(p->lum_xbar_erg_s >= 0.0)))
    return NBO_EINVAL;
  nbo_model *m = (nbo_model *)calloc(1, sizeof(nbo_model));
  m->p = *p;
  m->nf = p->n_flavor;
  m->ncomp = (m->nf == 2) ? 3 : 8;
  m->nsc = (m->nf == 2) ? 3 : 6;
  m->NE = p->n_energy;
  m->NU = p->n_u;
  /* species rows: two tracked (nu_e-born, anti-nu_e-born) or every flavour explicitly */
  if (!p->species4) {
    m->ns = 2;
    m->anti[0] = 0; m->init_flav[0] = 0;
    m->anti[1] = 1; m->init_flav[1] = 0;
  } else {
    m->ns = 2 * m->nf;
    for (int s = 0; s < m->ns; ++s) { m->anti[s] = s / m->nf; m->init_flav[s] = s % m->nf; }
  }
  m->ext = p->n_phi >= 1;
  m->NP = m->ext ? p->n_phi : 1;
  m->nb = (int64_t)m->ns * m->NU * m->NP * m->NE;
  m->cphi = (double *)malloc(sizeof(double) * m->NP);
  m->sphi = (double *)malloc(sizeof(double) * m->NP);
  /* azimuthal bin midpoints phi_p = 2 pi (p + 1/2) / n_phi; for even n_phi the second half
   * is the first half turned by pi with the signs flipped exactly, so that the azimuthal
   * sums of an axially symmetric state vanish exactly */
  for (int64_t q = 0; q < m->NP; ++q) {
    if (m->NP % 2 == 0 && q >= m->NP / 2) {
      m->cphi[q] = -m->cphi[q - m->NP / 2];
      m->sphi[q] = -m->sphi[q - m->NP / 2];
    } else {
      const double ph = (2.0 * PI_D) * (((double)q + 0.5) / (double)m->NP);
      m->cphi[q] = cos(ph);
      m->sphi[q] = sin(ph);
    }
  }
  m->dE = (p->e_max_mev - p->e_min_mev) / (double)m->NE;
  m->du = 1.0 / (double)m->NU;
  m->h = (p->r_end_km - p->r_start_km) / (double)p->n_steps;
  m->R = p->r_nu_km;
  const double s2gf = sqrt2gf_km_cm3();
  m->lam0 = s2gf * p->n0_cm3;
  const double rcm = m->R * 1.0e5;
  m->kappa0 = s2gf / (((2.0 * PI_D) * (rcm * rcm)) * C_CM_S);
  m->E = (double *)malloc(sizeof(double) * m->NE);
  m->w = (double *)malloc(sizeof(double) * m->NE * m->ns);
  m->bv = (double *)malloc(sizeof(double) * m->NE * (m->nf == 2 ? 2 : 6));
  m->ek = (double *)malloc(sizeof(double) * m->NE);
  m->X = (double *)malloc(sizeof(double) * m->nb * m->nsc);
  m->Y = (double *)malloc(sizeof(double) * m->nb * m->nsc);
  /* number luminosities N = L / <E>, <E> = T F3/F2 (Fermi-Dirac, zero chemical potential) */
  /* [3]: anti-nu_x, its own spectrum or that of nu_x */
  double N[4], T[4];
  for (int a = 0; a < 3; ++a) T[a] = p->temp_mev[a];
  T[3] = (p->temp_xbar_mev != 0.0) ? p->temp_xbar_mev : p->temp_mev[2];
  const double Lxb = (p->temp_xbar_mev != 0.0) ? p->lum_xbar_erg_s : p->lum_erg_s[2];
  for (int a = 0; a < 3; ++a) N[a] = p->lum_erg_s[a] * ERG_MEV / ((T[a] * F3_0) / F2_0);
  N[3] = Lxb * ERG_MEV / ((T[3] * F3_0) / F2_0);
  /* extended model: the azimuthal average (1/2pi) int dphi' becomes the mean over bins */
  const double pref = m->ext ? ((m->kappa0 * m->du) * m->dE) * (1.0 / (double)m->NP)
                             : (m->kappa0 * m->du) * m->dE;
  for (int64_t k = 0; k < m->NE; ++k) {
    const double E = p->e_min_mev + ((double)k + 0.5) * m->dE;
    m->E[k] = E;
    const double fe = fermi_dirac(E, p->temp_mev[0]);
    const double fb = fermi_dirac(E, p->temp_mev[1]);
    const double fx = fermi_dirac(E, p->temp_mev[2]);
    const double fxb = fermi_dirac(E, T[3]);
    if (!p->species4) {
      /* heavy-flavour-born states are I - rho_e (unitarity), so they enter with -N_x f_x
       * (antineutrinos: -N_xbar f_xbar) */
      m->w[0 * m->NE + k] = pref * (N[0] * fe - N[2] * fx);
      m->w[1 * m->NE + k] = pref * (N[1] * fb - N[3] * fxb);
    } else {
      for (int s = 0; s < m->ns; ++s) {
        const int a = m->anti[s], fl = m->init_flav[s];
        double Nf;
        if (fl == 0) Nf = a ? N[1] * fb : N[0] * fe;
        else Nf = a ? N[3] * fxb : N[2] * fx;
        m->w[s * m->NE + k] = pref * Nf;
      }
    }
    if (m->nf == 2) {
      const double om = (VAC_K * p->dm2_ev2[0]) / E;
      const double s2 = sin(2.0 * p->theta[0]), c2 = cos(2.0 * p->theta[0]);
      m->bv[2 * k + 0] = (2.0 * om) * s2;      /* B_vac = (2w sin2t, 0, -2w cos2t) */
      m->bv[2 * k + 1] = -((2.0 * om) * c2);
    } else {
      const double c12 = cos(p->theta[0]), s12 = sin(p->theta[0]);
      const double c13 = cos(p->theta[1]), s13 = sin(p->theta[1]);
      const double c23 = cos(p->theta[2]), s23 = sin(p->theta[2]);
      const double U[3][3] = {
          {c12 * c13, s12 * c13, s13},
          {-(s12 * c23) - (c12 * s23) * s13, c12 * c23 - (s12 * s23) * s13, s23 * c13},
          {s12 * s23 - (c12 * c23) * s13, -(c12 * s23) - (s12 * c23) * s13, c23 * c13}};
      const double w2 = ((2.0 * VAC_K) * p->dm2_ev2[0]) / E; /* dm21 / 2E */
      const double w3 = ((2.0 * VAC_K) * p->dm2_ev2[1]) / E; /* dm31 / 2E */
      const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
      for (int e = 0; e < 6; ++e) {
        m->bv[6 * k + e] = (U[ia[e]][1] * U[ib[e]][1]) * w2 + (U[ia[e]][2] * U[ib[e]][2]) * w3;
        m->v0[e] = (U[ia[e]][1] * U[ib[e]][1]) * ((2.0 * VAC_K) * p->dm2_ev2[0]) +
                   (U[ia[e]][2] * U[ib[e]][2]) * ((2.0 * VAC_K) * p->dm2_ev2[1]);
      }
      m->ek[k] = 1.0 / E;
    }
  }
  /* fixed-point scales: every beam contribution |w rho~| 2^e1 < 2^50 (converted by rounding,
   * and 32 of them add up far inside a signed 64-bit integer) and every angle term of J0
   * times 2^e0 < 2^62 */
  double wmax = 0.0;
  for (int64_t i = 0; i < m->NE * m->ns; ++i)
    if (fabs(m->w[i]) > wmax) wmax = fabs(m->w[i]);
  if (!(wmax > 0.0)) wmax = 1.0;
  int ex;
  frexp(wmax, &ex);
  m->e1 = 50 - ex;
  const double qs = m->R / p->r_start_km;
  const double cmin = sqrt(1.0 - u_of(m, m->NU - 1) * (qs * qs));
  const double b0 = (wmax * (double)m->NE) * (1.0 / cmin);
  frexp(b0, &ex);
  m->e0 = 61 - ex;
  m->s1 = ldexp(1.0, m->e1); m->p2e1 = ldexp(1.0, -m->e1);
  m->s0 = ldexp(1.0, m->e0); m->p2e0 = ldexp(1.0, -m->e0);
  nbo_reset(m);
  *out = m;
  return NBO_OK;
}

void nbo_destroy(nbo_model *m) {
  if (!m) return;
  free(m->E); free(m->w); free(m->bv); free(m->ek); free(m->X); free(m->Y); free(m->cphi); free(m->sphi);
  free(m);
}

int64_t nbo_n_beams(const nbo_model *m) { return m->nb; }
int nbo_n_species(const nbo_model *m) { return m->ns; }
int nbo_state_comps(const nbo_model *m) { return m->nsc; }
int64_t nbo_step_index(const nbo_model *m) { return m->step; }

int nbo_reset(nbo_model *m) {
  for (int64_t b = 0; b < m->nb; ++b) {
    const int s = (int)(b / (m->NU * m->NP * m->NE));
    double *x = m->X + b * m->nsc;
    const int fl = m->init_flav[s];
    if (m->nf == 2) { x[0] = 0.0; x[1] = 0.0; x[2] = fl == 0 ? 1.0 : -1.0; }
    else { for (int c = 0; c < 6; ++c) x[c] = 0.0; x[2 * fl] = 1.0; }
  }
  m->step = 0;
  return NBO_OK;
}

/* rho~ of one beam: rho for neutrinos, -rho^* for antineutrinos (Eq. F), as the moment
 * components (2f: Bloch vector; 3f: rho_ee-rho_tt, rho_mm-rho_tt, Re/Im rho_em, rho_et, rho_mt). */
static double rho_tilde(const nbo_model *m, int s, const double *x, double *out) {
  const int a = m->anti[s];
  if (m->nf == 2) {
    out[0] = a ? -x[0] : x[0];
    out[1] = x[1];
    out[2] = a ? -x[2] : x[2];
    return fma(x[0], x[0], fma(x[1], x[1], x[2] * x[2]));
  }
  const cx p0 = cx_make(x[0], x[1]), p1 = cx_make(x[2], x[3]), p2 = cx_make(x[4], x[5]);
  const double n0 = cx_norm2(p0), n1 = cx_norm2(p1), n2 = cx_norm2(p2);
  const cx em = cx_mulc(p0, p1), et = cx_mulc(p0, p2), mt = cx_mulc(p1, p2);
  const double v[8] = {n0 - n2, n1 - n2, em.re, em.im, et.re, et.im, mt.re, mt.im};
  if (!a) {
    for (int c = 0; c < 8; ++c) out[c] = v[c];
  } else {
    out[0] = -v[0]; out[1] = -v[1];
    out[2] = -v[2]; out[3] = v[3];
    out[4] = -v[4]; out[5] = v[5];
    out[6] = -v[6]; out[7] = v[7];
  }
  return (n0 + n1) + n2;
}

/* J0 = sum_b g_b rho~_b / c_b(r), J1 = sum_b g_b rho~_b: the energy sum of each
 * (species, angle[, azimuth]) row is taken first, exactly in fixed point, then the angle
 * sum.  Extended model (Eq. F with the azimuthal moments): also
 * J_sc = sum_b g_b rho~_b sin(theta_b) cos(phi_b) / c_b and J_ss (sin(phi_b)), per row from
 * the row's energy sum like J0.  Jm[0..1] (bulb) or Jm[0..3] receive the moments. */
static int moments(const nbo_model *m, const double *X, double r, double (*Jm)[8]) {
  const radial g = radial_at(m, r);
  const int nc = m->ncomp;
  const int nm = m->ext ? 4 : 2;
  const int64_t nrow = (int64_t)m->ns * m->NU * m->NP;
  i128 *T = (i128 *)calloc((size_t)nrow * nm * nc, sizeof(i128));
  int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
  for (int64_t row = 0; row < nrow; ++row) {
    const int s = (int)(row / (m->NU * m->NP));
    const int64_t j = (row / m->NP) % m->NU, q = row % m->NP;
    const bgeo bg = geo_of(m, &g, j, q);
    const double ic = 1.0 / bg.c;
    i128 S[8] = {0};
    for (int64_t k = 0; k < m->NE; ++k) {
      const int64_t b = row * m->NE + k;
      double v[8];
      /* a state of squared norm 2 or more (NaN included) is a numerical failure */
      if (!(rho_tilde(m, s, X + b * m->nsc, v) < 2.0)) err = 1;
      const double ws = m->w[s * m->NE + k] * m->s1;
      for (int c = 0; c < nc; ++c) S[c] += fix_round(v[c], ws);
    }
    i128 *t = T + row * nm * nc;
    for (int c = 0; c < nc; ++c) {
      const double e = i128_to_double(S[c]) * m->p2e1;
      t[c] = to_fix(ic * e, m->s0, TWO62, &err);
      t[nc + c] = S[c];
      if (m->ext) {
        const double a = bg.sn * ic;
        t[2 * nc + c] = to_fix((a * bg.cp) * e, m->s0, TWO62, &err);
        t[3 * nc + c] = to_fix((a * bg.sp) * e, m->s0, TWO62, &err);
      }
    }
  }
  for (int i = 0; i < nm; ++i)
    for (int c = 0; c < nc; ++c) {
      i128 acc = 0;
      for (int64_t row = 0; row < nrow; ++row) acc += T[(row * nm + i) * nc + c];
      Jm[i][c] = i128_to_double(acc) * (i == 1 ? m->p2e1 : m->p2e0);
    }
  free(T);
  return err ? NBO_ENUMERIC : NBO_OK;
}

/* The neutrino-neutrino term of a beam: mu (J0 - c J1) in the bulb model (Eq. Hnu with
 * 1 - v.v' = 1 - c c'); the extended model adds - mu sin(theta) (cos(phi) J_sc +
 * sin(phi) J_ss) from the azimuthal part of 1 - v.v'. */
static inline double nunu_of(const nbo_model *m, const radial *g, const bgeo *bg,
                             const double (*Jm)[8], int i) {
  if (!m->ext) return g->mu * (Jm[0][i] - bg->c * Jm[1][i]);
  return g->mu * ((Jm[0][i] - bg->c * Jm[1][i]) - bg->sn * (bg->cp * Jm[2][i] + bg->sp * Jm[3][i]));
}

/* Hamiltonian of beam (s, k) with geometry bg (Eq. eom):
 * nu:   H_vac + lam E_ee + nn
 * nubar: H_vac - lam E_ee - nn^*                                                      */
static void beam_B2(const nbo_model *m, int s, int64_t k, const radial *g, const bgeo *bg,
                    const double (*Jm)[8], double B[3]) {
  const double nx = nunu_of(m, g, bg, Jm, 0);
  const double ny = nunu_of(m, g, bg, Jm, 1);
  const double nz = nunu_of(m, g, bg, Jm, 2);
  const double bx = m->bv[2 * k], bz = m->bv[2 * k + 1];
  if (!m->anti[s]) { B[0] = bx + nx; B[1] = ny; B[2] = (bz + g->lam) + nz; }
  else { B[0] = bx - nx; B[1] = ny; B[2] = (bz - g->lam) - nz; }
}
static void beam_H3(const nbo_model *m, int s, int64_t k, const radial *g, const bgeo *bg,
                    const double (*Jm)[8], herm3 *H) {
  double nn[8];
  for (int i = 0; i < 8; ++i) nn[i] = nunu_of(m, g, bg, Jm, i);
  const double *v = m->bv + 6 * k;
  if (!m->anti[s]) {
    H->d[0] = (v[0] + g->lam) + nn[0];
    H->d[1] = v[1] + nn[1];
    H->d[2] = v[2];
    H->o[0] = cx_make(v[3] + nn[2], nn[3]);
    H->o[1] = cx_make(v[4] + nn[4], nn[5]);
    H->o[2] = cx_make(v[5] + nn[6], nn[7]);
  } else {
    H->d[0] = (v[0] - g->lam) - nn[0];
    H->d[1] = v[1] - nn[1];
    H->d[2] = v[2];
    H->o[0] = cx_make(v[3] - nn[2], nn[3]);
    H->o[1] = cx_make(v[4] - nn[4], nn[5]);
    H->o[2] = cx_make(v[5] - nn[6], nn[7]);
  }
}

/* Scaled stage generator of beam b at radius g: 2f f = (h/c) B (3f: row_gen3 below). */
static void stage_f2h(const nbo_model *m, int64_t b, const radial *g, const double (*Jm)[8],
                      double h, double f[3]) {
  int s;
  int64_t j, q, k;
  beam_of(m, b, &s, &j, &q, &k);
  const bgeo bg = geo_of(m, g, j, q);
  const double hc = h / bg.c;
  double B[3];
  beam_B2(m, s, k, g, &bg, Jm, B);
  f[0] = hc * B[0]; f[1] = hc * B[1]; f[2] = hc * B[2];
}
/* the 2-flavour generator of the fixed step h = (r_end - r_start) / n_steps */
static void stage_f2(const nbo_model *m, int64_t b, const radial *g, const double (*Jm)[8],
                     double f[3]) {
  stage_f2h(m, b, g, Jm, m->h, f);
}

/* Renormalisation after a step: a unitary step leaves the squared norm at 1 + d with d at
 * rounding level, so one Newton step for 1/sqrt(n2) from 1, 1.5 - n2/2, equals 1/sqrt(n2)
 * to within 3 d^2 / 8 (a state set far from unit norm converges to it quadratically over
 * the following steps; one with n2 >= 2 fails the moments' state check). */
static void renorm2(double *P) {
  const double n2 = (P[0] * P[0] + P[1] * P[1]) + P[2] * P[2];
  const double inv = fma(-0.5, n2, 1.5);
  P[0] = P[0] * inv; P[1] = P[1] * inv; P[2] = P[2] * inv;
}
static void renorm3(double *x) {
  const double n2 = (cx_norm2(cx_make(x[0], x[1])) + cx_norm2(cx_make(x[2], x[3]))) +
                    cx_norm2(cx_make(x[4], x[5]));
  const double inv = fma(-0.5, n2, 1.5);
  for (int c = 0; c < 6; ++c) x[c] = x[c] * inv;
}

static inline void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static void apply3(const herm3 *K, const double *x, double *y) {
  const cx ps[3] = {cx_make(x[0], x[1]), cx_make(x[2], x[3]), cx_make(x[4], x[5])};
  cx o[3];
  exp3_apply(K, ps, o);
  for (int c = 0; c < 3; ++c) { y[2 * c] = o[c].re; y[2 * c + 1] = o[c].im; }
}

/* Three-flavour stage generators by linearity.  Stage i's generator of a beam of energy
 * bin k is K_i = a_i (V_k + M_i): a_i = h / c_i with c_i = cos(theta) at the stage radius,
 * V_k = e_k V0 the vacuum Hamiltonian of the bin (e_k = 1 / E_k), M_i the matter and nu-nu
 * part, which is the same for every energy of a (species, angle) row.  Every generator the
 * step exponentiates is affine in V_k: with
 *   i[K_1, K_i] = a_1 a_i i[V_k + M_1, M_i - M_1] = a_1 a_i (e_k i[V0, D] + i[M_1, D]),
 * D = M_i - M_1, each is G = alpha V_k + e_k P + Q with alpha, P, Q fixed per row:
 *   K1/2                alpha = a1/2, P = 0, Q = (a1/2) M1
 *   K3                  alpha = am,   P = 0, Q = am M3
 *   K2/2 + i[K1,K2]/8   alpha = am/2, P = c i[V0, D], Q = (am/2) M2 + c i[M1, D],
 *                       c = a1 am / 8, D = M2 - M1
 *   Theta               alpha = (a1 + 2 am + 2 am + a4)/6, P = c i[V0, D], Q = S/6 + c i[M1, D],
 *                       c = a1 a4 / 12, D = M4 - M1, S = a1 M1 + 2 am M2 + 2 am M3 + a4 M4
 * (am: stages 2 and 3 share the radius r + h/2).  The step's error estimate takes
 * Theta - K2 = (alpha - am) V_k + e_k P + (Q - am M2).  Hermitian 3x3 matrices are
 * handled here as 9 reals: d0 d1 d2, then re and im of the (0,1), (0,2), (1,2) entries. */
static void h3_to9(const herm3 *h, double o[9]) {
  o[0] = h->d[0]; o[1] = h->d[1]; o[2] = h->d[2];
  for (int i = 0; i < 3; ++i) { o[3 + 2 * i] = h->o[i].re; o[4 + 2 * i] = h->o[i].im; }
}
static herm3 h3_from9(const double o[9]) {
  herm3 h;
  h.d[0] = o[0]; h.d[1] = o[1]; h.d[2] = o[2];
  for (int i = 0; i < 3; ++i) h.o[i] = cx_make(o[3 + 2 * i], o[4 + 2 * i]);
  return h;
}
/* M of species s at stage radius g: lam E_ee + nn (nu), -(lam E_ee + nn^*) (nubar) */
static void matter_M3(const nbo_model *m, int s, const radial *g, const bgeo *bg,
                      const double (*Jm)[8], double M[9]) {
  double nn[8];
  for (int i = 0; i < 8; ++i) nn[i] = nunu_of(m, g, bg, Jm, i);
  const double sg = m->anti[s] ? -1.0 : 1.0;
  M[0] = sg * (g->lam + nn[0]);
  M[1] = sg * nn[1];
  M[2] = 0.0;
  for (int i = 0; i < 3; ++i) { M[3 + 2 * i] = sg * nn[2 + 2 * i]; M[4 + 2 * i] = nn[3 + 2 * i]; }
}
typedef struct { double alpha, alphaE; double P[9], Q[9], QE[9]; } lingen3;
/* alpha V_k (+ e_k P) + Q for the six vacuum entries of bin k (v) */
static herm3 lin3(double alpha, const double *P, const double *Q, const double *v, double ek) {
  double o[9];
  for (int i = 0; i < 3; ++i) o[i] = fma(alpha, v[i], P ? fma(ek, P[i], Q[i]) : Q[i]);
  for (int i = 0; i < 3; ++i) {
    const int r = 3 + 2 * i, im = 4 + 2 * i;
    o[r] = fma(alpha, v[3 + i], P ? fma(ek, P[r], Q[r]) : Q[r]);
    o[im] = P ? fma(ek, P[im], Q[im]) : Q[im];
  }
  return h3_from9(o);
}
/* The row constants of generator `kind` (1: K1/2, 2: K2/2 + i[K1,K2]/8, 3: K3, 4: Theta)
 * for the row of beam b; J[i] are the stage moments. */
static void row_gen3(const nbo_model *m, int64_t b, int kind, const radial *g0, const radial *gm,
                     const radial *g1, const double (*J)[4][8], double h, lingen3 *L) {
  int s;
  int64_t j, q, k;
  beam_of(m, b, &s, &j, &q, &k);
  const bgeo b0 = geo_of(m, g0, j, q), bm = geo_of(m, gm, j, q), b1 = geo_of(m, g1, j, q);
  const double a1 = h / b0.c, am = h / bm.c, a4 = h / b1.c;
  double M1[9], M2[9], M3[9], M4[9];
  if (kind != 3) matter_M3(m, s, g0, &b0, J[0], M1);
  if (kind == 2 || kind == 4) matter_M3(m, s, gm, &bm, J[1], M2);
  if (kind >= 3) matter_M3(m, s, gm, &bm, J[2], M3);
  if (kind == 4) matter_M3(m, s, g1, &b1, J[3], M4);
  if (kind == 1 || kind == 3) {
    L->alpha = (kind == 1) ? 0.5 * a1 : am;
    for (int i = 0; i < 9; ++i) L->Q[i] = L->alpha * ((kind == 1) ? M1[i] : M3[i]);
    return;
  }
  const double *Mi = (kind == 2) ? M2 : M4;
  double D[9];
  for (int i = 0; i < 9; ++i) D[i] = Mi[i] - M1[i];
  herm3 V0, Dh = h3_from9(D), M1h = h3_from9(M1);
  V0.d[0] = m->v0[0]; V0.d[1] = m->v0[1]; V0.d[2] = m->v0[2];
  for (int i = 0; i < 3; ++i) V0.o[i] = cx_make(m->v0[3 + i], 0.0);
  const herm3 R1h = h3_icomm(&V0, &Dh), R2h = h3_icomm(&M1h, &Dh);
  double R1[9], R2[9];
  h3_to9(&R1h, R1);
  h3_to9(&R2h, R2);
  if (kind == 2) {
    const double c = (a1 * am) * 0.125;
    L->alpha = 0.5 * am;
    for (int i = 0; i < 9; ++i) {
      L->P[i] = c * R1[i];
      L->Q[i] = fma(L->alpha, M2[i], c * R2[i]);
    }
    return;
  }
  const double c = (a1 * a4) * (1.0 / 12.0), a2 = 2.0 * am;
  L->alpha = (((a1 + a2) + a2) + a4) * (1.0 / 6.0);
  L->alphaE = L->alpha - am;
  for (int i = 0; i < 9; ++i) {
    const double S = fma(a4, M4[i], fma(a2, M3[i], fma(a2, M2[i], a1 * M1[i])));
    L->P[i] = c * R1[i];
    L->Q[i] = fma(S, 1.0 / 6.0, c * R2[i]);
    L->QE[i] = fma(-am, M2[i], L->Q[i]);
  }
}
/* generator `kind` of beam b (its row constants, then the bin's vacuum entries) */
static herm3 gen3_lin(const nbo_model *m, int64_t b, int kind, const radial *g0, const radial *gm,
                      const radial *g1, const double (*J)[4][8], double h, herm3 *Ediff) {
  lingen3 L;
  row_gen3(m, b, kind, g0, gm, g1, J, h, &L);
  const int64_t k = b % m->NE;
  const double *v = m->bv + 6 * k;
  const int wp = (kind == 2 || kind == 4);
  if (Ediff) *Ediff = lin3(L.alphaE, L.P, L.QE, v, m->ek[k]);
  return lin3(L.alpha, wp ? L.P : NULL, L.Q, v, m->ek[k]);
}

/* One RKMK4 step (see the file header) from the state X at r0 over the step length h,
 * with stage radii r0, rm = r0 + h/2 and r1 = r0 + h (r1 passed separately so that the
 * fixed-step grid r_n = r_start + n h is reproduced exactly).  The new state goes to Xout
 * (which may be X).  If emax is not NULL it receives the embedded error estimate of the
 * step: the largest over beams of |Theta - F_2|^2, the squared distance between the
 * order-4 generator and the generator of the exponential midpoint rule (order 2) built
 * from the same stages (3 flavours: traceless part, Frobenius norm), with the low 16 bits
 * of its binary representation cleared. */
static int rkmk4_step(nbo_model *m, const double *X, double r0, double rm, double r1, double h,
                      double *Xout, double *emax) {
  const radial g0 = radial_at(m, r0), gm = radial_at(m, rm), g1 = radial_at(m, r1);
  double J[4][4][8];
  const double (*CJ)[4][8] = (const double (*)[4][8])J;
  int st = moments(m, X, r0, J[0]);
  const int64_t nb = m->nb;
  const int nsc = m->nsc;
  double *eb = emax ? (double *)malloc(sizeof(double) * nb) : NULL;
  /* stage 2 */
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    const double *x = X + b * nsc;
    double *y = m->Y + b * nsc;
    if (m->nf == 2) {
      double f1[3], o[3];
      stage_f2h(m, b, &g0, J[0], h, f1);
      o[0] = 0.5 * f1[0]; o[1] = 0.5 * f1[1]; o[2] = 0.5 * f1[2];
      rotate2(o, x, y);
    } else {
      const herm3 O = gen3_lin(m, b, 1, &g0, &gm, &g1, CJ, h, NULL);   /* K1/2 */
      apply3(&O, x, y);
    }
  }
  st |= moments(m, m->Y, rm, J[1]);
  /* stage 3 */
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    const double *x = X + b * nsc;
    double *y = m->Y + b * nsc;
    if (m->nf == 2) {
      double f1[3], f2[3], cr[3], o[3];
      stage_f2h(m, b, &g0, J[0], h, f1);
      stage_f2h(m, b, &gm, J[1], h, f2);
      cross3(f1, f2, cr);
      for (int c = 0; c < 3; ++c) o[c] = 0.5 * f2[c] - 0.125 * cr[c];
      rotate2(o, x, y);
    } else {
      const herm3 O = gen3_lin(m, b, 2, &g0, &gm, &g1, CJ, h, NULL);   /* K2/2 + i[K1,K2]/8 */
      apply3(&O, x, y);
    }
  }
  st |= moments(m, m->Y, rm, J[2]);
  /* stage 4 */
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    const double *x = X + b * nsc;
    double *y = m->Y + b * nsc;
    if (m->nf == 2) {
      double f3[3];
      stage_f2h(m, b, &gm, J[2], h, f3);
      rotate2(f3, x, y);
    } else {
      const herm3 K3 = gen3_lin(m, b, 3, &g0, &gm, &g1, CJ, h, NULL);
      apply3(&K3, x, y);
    }
  }
  st |= moments(m, m->Y, r1, J[3]);
  /* final update */
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    const double *x = X + b * nsc;
    double *xo = Xout + b * nsc;
    if (m->nf == 2) {
      double f1[3], f2[3], f3[3], f4[3], cr[3], th[3], y[3];
      stage_f2h(m, b, &g0, J[0], h, f1);
      stage_f2h(m, b, &gm, J[1], h, f2);
      stage_f2h(m, b, &gm, J[2], h, f3);
      stage_f2h(m, b, &g1, J[3], h, f4);
      cross3(f1, f4, cr);
      for (int c = 0; c < 3; ++c)
        th[c] = (((f1[c] + 2.0 * f2[c]) + 2.0 * f3[c]) + f4[c]) * (1.0 / 6.0) - cr[c] * (1.0 / 12.0);
      if (eb) {
        const double d0 = th[0] - f2[0], d1 = th[1] - f2[1], d2 = th[2] - f2[2];
        eb[b] = (d0 * d0 + d1 * d1) + d2 * d2;
      }
      rotate2(th, x, y);
      if (m->p.renorm) renorm2(y);
      xo[0] = y[0]; xo[1] = y[1]; xo[2] = y[2];
    } else {
      herm3 Ed;
      const herm3 T = gen3_lin(m, b, 4, &g0, &gm, &g1, CJ, h, eb ? &Ed : NULL);   /* Theta */
      if (eb) {
        /* |Theta - K2|^2: traceless part, Frobenius norm */
        double a[3], o2[3];
        const double tr = ((Ed.d[0] + Ed.d[1]) + Ed.d[2]) * (1.0 / 3.0);
        for (int i = 0; i < 3; ++i) a[i] = Ed.d[i] - tr;
        for (int i = 0; i < 3; ++i) o2[i] = Ed.o[i].re * Ed.o[i].re + Ed.o[i].im * Ed.o[i].im;
        eb[b] = ((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]) + 2.0 * ((o2[0] + o2[1]) + o2[2]);
      }
      double y[6];
      apply3(&T, x, y);
      if (m->p.renorm) renorm3(y);
      for (int c = 0; c < 6; ++c) xo[c] = y[c];
    }
  }
  if (eb) {
    double e = 0.0;
    for (int64_t b = 0; b < nb; ++b)
      if (eb[b] > e) e = eb[b];
    uint64_t bits;
    memcpy(&bits, &e, 8);
    bits &= ~(uint64_t)0xffff;
    memcpy(emax, &bits, 8);
    free(eb);
  }
  return st;
}

/* One step of the fixed grid r_n = r_start + n h, in place. */
static int step_rkmk4(nbo_model *m) {
  const double rs = m->p.r_start_km, h = m->h;
  const double r0 = rs + (double)m->step * h;
  const double rm = r0 + 0.5 * h;
  const double r1 = rs + (double)(m->step + 1) * h;
  const int st = rkmk4_step(m, m->X, r0, rm, r1, h, m->X, NULL);
  m->step += 1;
  return st;
}

/* The error estimate of one step of length h from the current state and step, without
 * advancing (for the estimator's pins). */
int nbo_step_error(nbo_model *m, double h, double *E) {
  if (!m || !(h > 0.0) || !E) return NBO_EINVAL;
  const double r0 = m->p.r_start_km + (double)m->step * m->h;
  double *Xs = (double *)malloc(sizeof(double) * (size_t)m->nb * (size_t)m->nsc);
  const int st = rkmk4_step(m, m->X, r0, r0 + 0.5 * h, r0 + h, h, Xs, E);
  free(Xs);
  return st ? NBO_ENUMERIC : NBO_OK;
}

/* Adaptive step-size control on top of the RKMK4 step (the paper integrates with an
 * adaptive step size, Sec. 3.4; the controller below is this library's own, with
 * power-of-two step changes so that both implementations take identical decisions):
 *   a step of length h from r is accepted if its error estimate E <= tol^2; the state
 *   and r advance, and h doubles (up to h_max) if E <= tol^2 / 128, i.e. when the doubled
 *   step's estimate, which grows as h^6 (a factor 64), is expected to pass with a margin
 *   of 2;
 *   a rejected step is retried from the same state with h / 2.
 * The last step is shortened to end exactly at r_end.  The first step length is the
 * model's (r_end - r_start) / n_steps; the run fails if h falls below 2^-40 of it or the
 * attempts exceed max_attempts.  The model must be at its start (step 0); it ends at
 * r_end with its step index set to n_steps. */
int nbo_run_adaptive(nbo_model *m, double tol, double h_max, int64_t max_attempts,
                     int64_t *accepted, int64_t *rejected, double *h_last) {
  if (!m || !(tol > 0.0) || max_attempts < 1 || m->step != 0 || m->p.integrator != 0)
    return NBO_EINVAL;
  const double r_end = m->p.r_end_km;
  double r = m->p.r_start_km, h = m->h;
  const double hmin = ldexp(m->h, -40);
  const double hmax = (h_max > 0.0) ? h_max : (r_end - r);
  const double tol2 = tol * tol, grow = tol2 * (1.0 / 128.0);
  const size_t bytes = sizeof(double) * (size_t)m->nb * (size_t)m->nsc;
  double *Xn = (double *)malloc(bytes);
  int64_t acc = 0, rej = 0, att = 0;
  int st = NBO_OK;
  for (;;) {
    const int last = (r + h >= r_end);
    const double hs = last ? r_end - r : h;
    const double r1 = last ? r_end : r + hs;
    double E = 0.0;
    if (rkmk4_step(m, m->X, r, r + 0.5 * hs, r1, hs, Xn, &E)) { st = NBO_ENUMERIC; break; }
    ++att;
    if (E <= tol2) {
      double *t = m->X; m->X = Xn; Xn = t;
      r = r1;
      ++acc;
      if (E <= grow && 2.0 * h <= hmax) h = 2.0 * h;
      if (last) break;
    } else {
      ++rej;
      h = 0.5 * h;
      if (h < hmin) { st = NBO_ESTEP; break; }
    }
    if (att >= max_attempts) { st = NBO_ESTEP; break; }
  }
  free(Xn);
  if (st == NBO_OK) m->step = m->p.n_steps;
  if (accepted) *accepted = acc;
  if (rejected) *rejected = rej;
  if (h_last) *h_last = h;
  return st;
}

/* Right-hand side for plain RK4: 2f dP/dr = (1/c) B x P; 3f dpsi/dr = -(i/c) H psi. */
static int rhs(const nbo_model *m, const double *X, double r, double *D) {
  double Jm[4][8];
  int st = moments(m, X, r, Jm);
  const radial g = radial_at(m, r);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nb; ++b) {
    int s;
    int64_t j, q, k;
    beam_of(m, b, &s, &j, &q, &k);
    const bgeo bg = geo_of(m, &g, j, q);
    const double ic = 1.0 / bg.c;
    const double *x = X + b * m->nsc;
    double *d = D + b * m->nsc;
    if (m->nf == 2) {
      double B[3], cr[3];
      beam_B2(m, s, k, &g, &bg, (const double (*)[8])Jm, B);
      cross3(B, x, cr);
      d[0] = ic * cr[0]; d[1] = ic * cr[1]; d[2] = ic * cr[2];
    } else {
      herm3 H;
      beam_H3(m, s, k, &g, &bg, (const double (*)[8])Jm, &H);
      const cx ps[3] = {cx_make(x[0], x[1]), cx_make(x[2], x[3]), cx_make(x[4], x[5])};
      for (int a = 0; a < 3; ++a) {
        const cx hp = cx_add(cx_add(cx_mul(h3_at(&H, a, 0), ps[0]), cx_mul(h3_at(&H, a, 1), ps[1])),
                             cx_mul(h3_at(&H, a, 2), ps[2]));
        d[2 * a] = ic * hp.im;
        d[2 * a + 1] = -(ic * hp.re);
      }
    }
  }
  return st;
}

static int step_rk4(nbo_model *m) {
  const double rs = m->p.r_start_km, h = m->h;
  const double r0 = rs + (double)m->step * h, rm = r0 + 0.5 * h;
  const double r1 = rs + (double)(m->step + 1) * h;
  const int64_t n = m->nb * m->nsc;
  double *k1 = (double *)malloc(sizeof(double) * n), *k2 = (double *)malloc(sizeof(double) * n);
  double *k3 = (double *)malloc(sizeof(double) * n), *k4 = (double *)malloc(sizeof(double) * n);
  int st = rhs(m, m->X, r0, k1);
  for (int64_t i = 0; i < n; ++i) m->Y[i] = m->X[i] + (0.5 * h) * k1[i];
  st |= rhs(m, m->Y, rm, k2);
  for (int64_t i = 0; i < n; ++i) m->Y[i] = m->X[i] + (0.5 * h) * k2[i];
  st |= rhs(m, m->Y, rm, k3);
  for (int64_t i = 0; i < n; ++i) m->Y[i] = m->X[i] + h * k3[i];
  st |= rhs(m, m->Y, r1, k4);
  for (int64_t i = 0; i < n; ++i)
    m->X[i] = m->X[i] + (h / 6.0) * (((k1[i] + 2.0 * k2[i]) + 2.0 * k3[i]) + k4[i]);
  if (m->p.renorm)
    for (int64_t b = 0; b < m->nb; ++b) {
      if (m->nf == 2) renorm2(m->X + b * 3);
      else renorm3(m->X + b * 6);
    }
  free(k1); free(k2); free(k3); free(k4);
  m->step += 1;
  return st;
}

int nbo_step(nbo_model *m, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    const int st = m->p.integrator ? step_rk4(m) : step_rkmk4(m);
    if (st) return NBO_ENUMERIC;
  }
  return NBO_OK;
}

int nbo_read_pee(const nbo_model *m, double *out) {
  for (int64_t b = 0; b < m->nb; ++b) {
    const double *x = m->X + b * m->nsc;
    out[b] = (m->nf == 2) ? 0.5 * (1.0 + x[2]) : cx_norm2(cx_make(x[0], x[1]));
  }
  return NBO_OK;
}

int nbo_get_state(const nbo_model *m, double *out) {
  for (int c = 0; c < m->nsc; ++c)
    for (int64_t b = 0; b < m->nb; ++b) out[c * m->nb + b] = m->X[b * m->nsc + c];
  return NBO_OK;
}
int nbo_set_state(nbo_model *m, const double *in, int64_t step) {
  if (step < 0) return NBO_EINVAL;
  for (int c = 0; c < m->nsc; ++c)
    for (int64_t b = 0; b < m->nb; ++b) m->X[b * m->nsc + c] = in[c * m->nb + b];
  m->step = step;
  return NBO_OK;
}

int nbo_tables(const nbo_model *m, double *out, int64_t cap) {
  const int nv = (m->nf == 2) ? 2 : 6;
  const int64_t need = m->NE + m->NE * m->ns + m->NE * nv + 7;
  if (cap < need) return NBO_EINVAL;
  int64_t o = 0;
  for (int64_t k = 0; k < m->NE; ++k) out[o++] = m->E[k];
  for (int64_t i = 0; i < m->NE * m->ns; ++i) out[o++] = m->w[i];
  for (int64_t i = 0; i < m->NE * nv; ++i) out[o++] = m->bv[i];
  out[o++] = m->lam0; out[o++] = m->kappa0; out[o++] = m->h;
  out[o++] = m->p2e1; out[o++] = m->p2e0; out[o++] = m->e1; out[o++] = m->e0;
  return NBO_OK;
}

int nbo_moments(const nbo_model *m, double r, double *j0, double *j1) {
  double Jm[4][8];
  const int st = moments(m, m->X, r, Jm);
  for (int c = 0; c < m->ncomp; ++c) { j0[c] = Jm[0][c]; j1[c] = Jm[1][c]; }
  return st;
}
int nbo_moments4(const nbo_model *m, double r, double *jm) {
  double Jm[4][8] = {{0}};
  const int st = moments(m, m->X, r, Jm);
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < m->ncomp; ++c) jm[i * m->ncomp + c] = Jm[i][c];
  return st;
}

int nbo_hamiltonian4(const nbo_model *m, double r, const double *jm, double *out) {
  double Jm[4][8] = {{0}};
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < m->ncomp; ++c) Jm[i][c] = jm[i * m->ncomp + c];
  const radial g = radial_at(m, r);
  for (int64_t b = 0; b < m->nb; ++b) {
    int s;
    int64_t j, q, k;
    beam_of(m, b, &s, &j, &q, &k);
    const bgeo bg = geo_of(m, &g, j, q);
    if (m->nf == 2) beam_B2(m, s, k, &g, &bg, (const double (*)[8])Jm, out + 3 * b);
    else {
      herm3 H;
      beam_H3(m, s, k, &g, &bg, (const double (*)[8])Jm, &H);
      double *o = out + 9 * b;
      o[0] = H.d[0]; o[1] = H.d[1]; o[2] = H.d[2];
      for (int i = 0; i < 3; ++i) { o[3 + 2 * i] = H.o[i].re; o[4 + 2 * i] = H.o[i].im; }
    }
  }
  return NBO_OK;
}

int nbo_hamiltonian(const nbo_model *m, double r, const double *j0, const double *j1,
                    double *out) {
  double jm[4 * 8] = {0};
  for (int c = 0; c < m->ncomp; ++c) { jm[c] = j0[c]; jm[m->ncomp + c] = j1[c]; }
  return nbo_hamiltonian4(m, r, jm, out);
}

int nbo_phi_table(const nbo_model *m, double *out) {
  if (!m->ext) return NBO_EINVAL;
  for (int64_t q = 0; q < m->NP; ++q) { out[q] = m->cphi[q]; out[m->NP + q] = m->sphi[q]; }
  return NBO_OK;
}

int nbo_cos_theta(const nbo_model *m, double r, double *out) {
  const radial g = radial_at(m, r);
  for (int64_t j = 0; j < m->NU; ++j) out[j] = c_of(&g, u_of(m, j));
  return NBO_OK;
}

void nbo_sincos(const double *x, int64_t n, double *s, double *c) {
  for (int64_t i = 0; i < n; ++i) sincos_spec(x[i], s + i, c + i);
}
void nbo_exp3_apply(const double *k9, const double *psi6, double *out6) {
  herm3 K;
  K.d[0] = k9[0]; K.d[1] = k9[1]; K.d[2] = k9[2];
  for (int i = 0; i < 3; ++i) K.o[i] = cx_make(k9[3 + 2 * i], k9[4 + 2 * i]);
  apply3(&K, psi6, out6);
}
void nbo_rotate(const double *x3, const double *p3, double *out3) { rotate2(x3, p3, out3); }
double nbo_fixed_sum(const double *v, int64_t n, int e) {
  i128 a = 0;
  int err = 0;
  const double sc = ldexp(1.0, e);
  for (int64_t i = 0; i < n; ++i) a += to_fix(v[i], sc, TWO62, &err);
  if (err) return NAN;
  return i128_to_double(a) * ldexp(1.0, -e);
}

/* The integer of every beam contribution fix_round(v[i], ws[i]) (tests). */
void nbo_fix_round(const double *v, const double *ws, int64_t n, int64_t *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = fix_round(v[i], ws[i]);
}

/* ------------------------------------------------------- single-angle solver */
/* All beams at one emission bin u = 1/2.  Then J0 = J1/c and the neutrino-neutrino
 * Hamiltonian reduces to mu (1/c - c) J1 for every beam: a direct E-only system. */
int nbo_single_angle_run(const nbo_params *pin, double *pee_out) {
  if (!pin || pin->n_flavor != 2) return NBO_EINVAL;
  nbo_params p = *pin;
  p.n_u = 1;
  p.species4 = 0;
  p.integrator = 0;
  nbo_model *m;
  int st = nbo_create(&p, &m);
  if (st) return st;
  const int64_t NE = m->NE;
  double *P = (double *)malloc(sizeof(double) * 2 * NE * 3);
  double *Y = (double *)malloc(sizeof(double) * 2 * NE * 3);
  for (int64_t i = 0; i < 2 * NE; ++i) { P[3 * i] = 0.0; P[3 * i + 1] = 0.0; P[3 * i + 2] = 1.0; }
  const double u = 0.5;
  int err = 0;
  for (int64_t n = 0; n < p.n_steps && !err; ++n) {
    const double rs = p.r_start_km, h = m->h;
    const double rr[4] = {rs + (double)n * h, rs + (double)n * h + 0.5 * h,
                          rs + (double)n * h + 0.5 * h, rs + (double)(n + 1) * h};
    double Jn[4][3];
    double *F = (double *)malloc(sizeof(double) * 4 * 2 * NE * 3);
    for (int st_i = 0; st_i < 4; ++st_i) {
      /* moments of the stage state */
      const double *src = (st_i == 0) ? P : Y;
      i128 S[3] = {0, 0, 0};
      for (int64_t i = 0; i < 2 * NE; ++i) {
        const int s = (int)(i / NE);
        const double *x = src + 3 * i;
        const double v[3] = {s ? -x[0] : x[0], x[1], s ? -x[2] : x[2]};
        if (!(fma(x[0], x[0], fma(x[1], x[1], x[2] * x[2])) < 2.0)) err = 1;
        const double ws = m->w[i] * m->s1;
        for (int c = 0; c < 3; ++c) S[c] += fix_round(v[c], ws);
      }
      for (int c = 0; c < 3; ++c) Jn[st_i][c] = i128_to_double(S[c]) * m->p2e1;
      const radial g = radial_at(m, rr[st_i]);
      const double c = sqrt(1.0 - u * g.q2);
      const double geo = g.mu * (1.0 / c - c);
      for (int64_t i = 0; i < 2 * NE; ++i) {
        const int s = (int)(i / NE);
        const int64_t k = i % NE;
        const double nn[3] = {geo * Jn[st_i][0], geo * Jn[st_i][1], geo * Jn[st_i][2]};
        double B[3];
        if (!s) { B[0] = m->bv[2 * k] + nn[0]; B[1] = nn[1]; B[2] = (m->bv[2 * k + 1] + g.lam) + nn[2]; }
        else { B[0] = m->bv[2 * k] - nn[0]; B[1] = nn[1]; B[2] = (m->bv[2 * k + 1] - g.lam) - nn[2]; }
        double *f = F + (st_i * 2 * NE + i) * 3;
        for (int cc = 0; cc < 3; ++cc) f[cc] = (h / c) * B[cc];
        double o[3];
        const double *f1 = F + (0 * 2 * NE + i) * 3;
        if (st_i == 0) { for (int cc = 0; cc < 3; ++cc) o[cc] = 0.5 * f[cc]; }
        else if (st_i == 1) {
          double cr[3];
          cross3(f1, f, cr);
          for (int cc = 0; cc < 3; ++cc) o[cc] = 0.5 * f[cc] - 0.125 * cr[cc];
        } else if (st_i == 2) { for (int cc = 0; cc < 3; ++cc) o[cc] = f[cc]; }
        else {
          const double *f2 = F + (1 * 2 * NE + i) * 3, *f3 = F + (2 * 2 * NE + i) * 3;
          double cr[3];
          cross3(f1, f, cr);
          for (int cc = 0; cc < 3; ++cc)
            o[cc] = (((f1[cc] + 2.0 * f2[cc]) + 2.0 * f3[cc]) + f[cc]) * (1.0 / 6.0) - cr[cc] * (1.0 / 12.0);
        }
        double y[3];
        rotate2(o, P + 3 * i, y);
        if (st_i == 3) { renorm2(y); for (int cc = 0; cc < 3; ++cc) P[3 * i + cc] = y[cc]; }
        else for (int cc = 0; cc < 3; ++cc) Y[3 * i + cc] = y[cc];
      }
    }
    free(F);
  }
  for (int64_t i = 0; i < 2 * NE; ++i) pee_out[i] = 0.5 * (1.0 + P[3 * i + 2]);
  free(P); free(Y);
  nbo_destroy(m);
  return err ? NBO_ENUMERIC : NBO_OK;
}

/* ------------------------------------------------------------------- adjoint */
/* Reverse mode of the two-flavour RKMK4 integration.  The moment sums are treated as the
 * exact sums they represent (the fixed-point quantisation is below 2^-50 of the largest
 * term).  Notation of the forward step (file header): f_i = (h/c_i) B(r_i, J^(i)),
 * Y2 = R(f1/2)P, Y3 = R(Om3)P with Om3 = f2/2 - f1 x f2/8, Y4 = R(f3)P,
 * Theta = (f1 + 2f2 + 2f3 + f4)/6 - f1 x f4/12, P' = R(Theta)P, P_{n+1} = P'/|P'|.
 * For a rotation y = R(x)p: p-bar = R(-x) y-bar and x-bar = Jl(x)^T (y x y-bar), with the
 * left Jacobian of SO(3), Jl(x) = I + a [x]x + b [x]x^2, a = (1-cos t)/t^2,
 * b = (t - sin t)/t^3, t = |x|.  The parameters enter through the weights g (the three
 * luminosities), the vacuum term (theta_v) and lambda(r) (n0). */

static void jlt(const double x[3], const double v[3], double out[3]) {
  const double t2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
  const double t = sqrt(t2);
  double a, b;
  if (t < 0.05) {
    a = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
    b = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
  } else {
    const double sh = sin(0.5 * t);
    a = 2.0 * sh * sh / t2;
    b = (t - sin(t)) / (t2 * t);
  }
  double c1[3], c2[3];
  cross3(x, v, c1);
  cross3(x, c1, c2);
  for (int i = 0; i < 3; ++i) out[i] = v[i] - a * c1[i] + b * c2[i];
}

/* Forward quantities of step n from P_n: the four stage moment sets. */
static int step_moments(nbo_model *m, const double *X, int64_t n, double J[4][2][8]) {
  const double rs = m->p.r_start_km, h = m->h;
  const double r0 = rs + (double)n * h, rm = r0 + 0.5 * h, r1 = rs + (double)(n + 1) * h;
  const radial g0 = radial_at(m, r0), gm = radial_at(m, rm);
  int st = moments(m, X, r0, J[0]);
  for (int64_t b = 0; b < m->nb; ++b) {
    double f1[3], o[3];
    stage_f2(m, b, &g0, (const double (*)[8])J[0], f1);
    for (int c = 0; c < 3; ++c) o[c] = 0.5 * f1[c];
    rotate2(o, X + 3 * b, m->Y + 3 * b);
  }
  st |= moments(m, m->Y, rm, J[1]);
  for (int64_t b = 0; b < m->nb; ++b) {
    double f1[3], f2[3], cr[3], o[3];
    stage_f2(m, b, &g0, (const double (*)[8])J[0], f1);
    stage_f2(m, b, &gm, (const double (*)[8])J[1], f2);
    cross3(f1, f2, cr);
    for (int c = 0; c < 3; ++c) o[c] = 0.5 * f2[c] - 0.125 * cr[c];
    rotate2(o, X + 3 * b, m->Y + 3 * b);
  }
  st |= moments(m, m->Y, rm, J[2]);
  for (int64_t b = 0; b < m->nb; ++b) {
    double f3[3];
    stage_f2(m, b, &gm, (const double (*)[8])J[2], f3);
    rotate2(f3, X + 3 * b, m->Y + 3 * b);
  }
  st |= moments(m, m->Y, r1, J[3]);
  return st;
}

typedef struct {
  double *dGe, *dGb, *dGx;   /* d w / d L per energy bin (for the species they enter) */
  double *dbx, *dbz;         /* d B_vac / d theta_v per energy bin */
  double s2gf;
} adj_tables;

/* B-bar of one beam at radius g: returns its contribution to the moment adjoints
 * (J0-bar += mu S B-bar, J1-bar -= mu c S B-bar) and to theta_v-bar, n0-bar. */
static void b_adjoint(const nbo_model *m, const adj_tables *t, int s, int64_t k, const radial *g,
                      double c, const double Bb[3], double *J0b, double *J1b, double *gth,
                      double *gn0) {
  const double sg = m->anti[s] ? -1.0 : 1.0;
  const double SB[3] = {sg * Bb[0], Bb[1], sg * Bb[2]};
  for (int i = 0; i < 3; ++i) { J0b[i] += g->mu * SB[i]; J1b[i] -= g->mu * c * SB[i]; }
  *gth += Bb[0] * t->dbx[k] + Bb[2] * t->dbz[k];
  double qp = 1.0;
  for (int i = 0; i < m->p.ne_power; ++i) qp *= g->q;
  *gn0 += sg * Bb[2] * t->s2gf * qp;
}

/* Moment adjoint broadcast to beam b at radius g: y-bar += w S (J0b/c + J1b) and the
 * weight adjoint w-bar += (S y).(J0b/c + J1b). */
static void m_adjoint(const nbo_model *m, int s, int64_t k, double c, const double *J0b,
                      const double *J1b, const double y[3], double yb[3], double *wb) {
  const double sg = m->anti[s] ? -1.0 : 1.0;
  const double w = m->w[s * m->NE + k];
  const double v[3] = {J0b[0] / c + J1b[0], J0b[1] / c + J1b[1], J0b[2] / c + J1b[2]};
  const double Sv[3] = {sg * v[0], v[1], sg * v[2]};
  for (int i = 0; i < 3; ++i) yb[i] += w * Sv[i];
  *wb += (sg * y[0]) * v[0] + y[1] * v[1] + (sg * y[2]) * v[2];
}

static void add_rot_adjoint(const double x[3], double scale, const double yb[3], double pb[3]) {
  double mx[3] = {-x[0] * scale, -x[1] * scale, -x[2] * scale}, r[3];
  rotate2(mx, yb, r);
  for (int i = 0; i < 3; ++i) pb[i] += r[i];
}

/* One reverse step: Pb (in: adjoint of P_{n+1}; out: adjoint of P_n), wbar per beam
 * accumulated, parameter gradients accumulated. */
static void reverse_step(nbo_model *m, const adj_tables *t, const double *X, int64_t n,
                         double *Pb, double *wbar, double *gth, double *gn0, double *Tb,
                         double *F1b) {
  double J[4][2][8];
  step_moments(m, X, n, J);
  const double rs = m->p.r_start_km, h = m->h;
  const double r0 = rs + (double)n * h, rm = r0 + 0.5 * h, r1 = rs + (double)(n + 1) * h;
  const radial g0 = radial_at(m, r0), gm = radial_at(m, rm), g1 = radial_at(m, r1);
  double Jb[4][2][3];
  memset(Jb, 0, sizeof Jb);
  /* final update and f4 */
  for (int64_t b = 0; b < m->nb; ++b) {
    const int s = (int)(b / (m->NU * m->NE));
    const int64_t j = (b / m->NE) % m->NU, k = b % m->NE;
    const double u = u_of(m, j);
    double f1[3], f2[3], f3[3], f4[3], cr[3], th[3], Pp[3];
    stage_f2(m, b, &g0, (const double (*)[8])J[0], f1);
    stage_f2(m, b, &gm, (const double (*)[8])J[1], f2);
    stage_f2(m, b, &gm, (const double (*)[8])J[2], f3);
    stage_f2(m, b, &g1, (const double (*)[8])J[3], f4);
    cross3(f1, f4, cr);
    for (int c = 0; c < 3; ++c)
      th[c] = (((f1[c] + 2.0 * f2[c]) + 2.0 * f3[c]) + f4[c]) * (1.0 / 6.0) - cr[c] * (1.0 / 12.0);
    rotate2(th, X + 3 * b, Pp);
    double Ppb[3] = {Pb[3 * b], Pb[3 * b + 1], Pb[3 * b + 2]};
    if (m->p.renorm) {
      /* y = P (1.5 - |P|^2 / 2): P-bar = (1.5 - |P|^2 / 2) y-bar - P (P . y-bar) */
      const double sf = 1.5 - 0.5 * ((Pp[0] * Pp[0] + Pp[1] * Pp[1]) + Pp[2] * Pp[2]);
      const double d = Pp[0] * Ppb[0] + Pp[1] * Ppb[1] + Pp[2] * Ppb[2];
      for (int c = 0; c < 3; ++c) Ppb[c] = sf * Ppb[c] - Pp[c] * d;
    }
    double pbn[3] = {0, 0, 0}, om[3], thb[3];
    add_rot_adjoint(th, 1.0, Ppb, pbn);
    cross3(Pp, Ppb, om);
    jlt(th, om, thb);
    double c4[3], c1[3];
    cross3(f4, thb, c4);     /* f1-bar part */
    cross3(thb, f1, c1);     /* f4-bar part */
    double f4b[3];
    for (int c = 0; c < 3; ++c) {
      F1b[3 * b + c] = thb[c] / 6.0 - c4[c] / 12.0;
      f4b[c] = thb[c] / 6.0 - c1[c] / 12.0;
      Tb[3 * b + c] = thb[c];
      Pb[3 * b + c] = pbn[c];
    }
    const double c1g = c_of(&g1, u);
    const double Bb[3] = {(h / c1g) * f4b[0], (h / c1g) * f4b[1], (h / c1g) * f4b[2]};
    b_adjoint(m, t, s, k, &g1, c1g, Bb, Jb[3][0], Jb[3][1], gth, gn0);
  }
  /* stage 4: Y4 = R(f3) P */
  for (int64_t b = 0; b < m->nb; ++b) {
    const int s = (int)(b / (m->NU * m->NE));
    const int64_t j = (b / m->NE) % m->NU, k = b % m->NE;
    const double u = u_of(m, j);
    double f3[3], Y[3], Yb[3] = {0, 0, 0}, om[3], f3b[3];
    stage_f2(m, b, &gm, (const double (*)[8])J[2], f3);
    rotate2(f3, X + 3 * b, Y);
    m_adjoint(m, s, k, c_of(&g1, u), Jb[3][0], Jb[3][1], Y, Yb, &wbar[b]);
    add_rot_adjoint(f3, 1.0, Yb, Pb + 3 * b);
    cross3(Y, Yb, om);
    jlt(f3, om, f3b);
    for (int c = 0; c < 3; ++c) f3b[c] += Tb[3 * b + c] / 3.0;
    const double cm = c_of(&gm, u);
    const double Bb[3] = {(h / cm) * f3b[0], (h / cm) * f3b[1], (h / cm) * f3b[2]};
    b_adjoint(m, t, s, k, &gm, cm, Bb, Jb[2][0], Jb[2][1], gth, gn0);
  }
  /* stage 3: Y3 = R(Om3) P */
  for (int64_t b = 0; b < m->nb; ++b) {
    const int s = (int)(b / (m->NU * m->NE));
    const int64_t j = (b / m->NE) % m->NU, k = b % m->NE;
    const double u = u_of(m, j);
    double f1[3], f2[3], cr[3], o[3], Y[3], Yb[3] = {0, 0, 0}, om[3], ob[3];
    stage_f2(m, b, &g0, (const double (*)[8])J[0], f1);
    stage_f2(m, b, &gm, (const double (*)[8])J[1], f2);
    cross3(f1, f2, cr);
    for (int c = 0; c < 3; ++c) o[c] = 0.5 * f2[c] - 0.125 * cr[c];
    rotate2(o, X + 3 * b, Y);
    const double cm = c_of(&gm, u);
    m_adjoint(m, s, k, cm, Jb[2][0], Jb[2][1], Y, Yb, &wbar[b]);
    add_rot_adjoint(o, 1.0, Yb, Pb + 3 * b);
    cross3(Y, Yb, om);
    jlt(o, om, ob);
    double a1[3], a2[3], f2b[3];
    cross3(ob, f1, a1);      /* f2-bar: ob/2 - (ob x f1)/8 */
    cross3(f2, ob, a2);      /* f1-bar: -(f2 x ob)/8 */
    for (int c = 0; c < 3; ++c) {
      f2b[c] = 0.5 * ob[c] - a1[c] / 8.0 + Tb[3 * b + c] / 3.0;
      F1b[3 * b + c] -= a2[c] / 8.0;
    }
    const double Bb[3] = {(h / cm) * f2b[0], (h / cm) * f2b[1], (h / cm) * f2b[2]};
    b_adjoint(m, t, s, k, &gm, cm, Bb, Jb[1][0], Jb[1][1], gth, gn0);
  }
  /* stage 2: Y2 = R(f1/2) P */
  for (int64_t b = 0; b < m->nb; ++b) {
    const int s = (int)(b / (m->NU * m->NE));
    const int64_t j = (b / m->NE) % m->NU, k = b % m->NE;
    const double u = u_of(m, j);
    double f1[3], o[3], Y[3], Yb[3] = {0, 0, 0}, om[3], ob[3];
    stage_f2(m, b, &g0, (const double (*)[8])J[0], f1);
    for (int c = 0; c < 3; ++c) o[c] = 0.5 * f1[c];
    rotate2(o, X + 3 * b, Y);
    m_adjoint(m, s, k, c_of(&gm, u), Jb[1][0], Jb[1][1], Y, Yb, &wbar[b]);
    add_rot_adjoint(o, 1.0, Yb, Pb + 3 * b);
    cross3(Y, Yb, om);
    jlt(o, om, ob);
    for (int c = 0; c < 3; ++c) F1b[3 * b + c] += 0.5 * ob[c];
    const double c0 = c_of(&g0, u);
    const double Bb[3] = {(h / c0) * F1b[3 * b], (h / c0) * F1b[3 * b + 1], (h / c0) * F1b[3 * b + 2]};
    b_adjoint(m, t, s, k, &g0, c0, Bb, Jb[0][0], Jb[0][1], gth, gn0);
  }
  /* stage 1 moments: J^(1) = M(P_n) */
  for (int64_t b = 0; b < m->nb; ++b) {
    const int s = (int)(b / (m->NU * m->NE));
    const int64_t j = (b / m->NE) % m->NU, k = b % m->NE;
    m_adjoint(m, s, k, c_of(&g0, u_of(m, j)), Jb[0][0], Jb[0][1], X + 3 * b, Pb + 3 * b, &wbar[b]);
  }
}

int nbo_adjoint(nbo_model *m, int32_t ckpt, const double *dl_dpee, double *grad, double *loss,
                double *state_bar) {
  if (!m || m->nf != 2 || m->p.species4 || m->p.integrator || m->ext || m->p.temp_xbar_mev != 0.0 ||
      ckpt < 1)
    return NBO_EINVAL;
  const int64_t n0 = m->step, N = m->p.n_steps;
  const int64_t nseg = (N - n0 + ckpt - 1) / ckpt;
  const int64_t ns = m->nb * 3;
  double *ck = (double *)malloc(sizeof(double) * ns * (size_t)(nseg > 0 ? nseg : 1));
  double *fin = (double *)malloc(sizeof(double) * ns);
  double *tape = (double *)malloc(sizeof(double) * ns * (size_t)ckpt);
  double *Pb = (double *)calloc((size_t)ns, sizeof(double));
  double *Tb = (double *)calloc((size_t)ns, sizeof(double));
  double *F1b = (double *)calloc((size_t)ns, sizeof(double));
  double *wbar = (double *)calloc((size_t)m->nb, sizeof(double));
  int st = 0;
  /* forward pass, keeping the state at the start of every segment */
  for (int64_t sgi = 0; sgi < nseg; ++sgi) {
    memcpy(ck + sgi * ns, m->X, sizeof(double) * ns);
    const int64_t len = (sgi == nseg - 1) ? (N - n0) - sgi * ckpt : ckpt;
    st |= nbo_step(m, len);
  }
  memcpy(fin, m->X, sizeof(double) * ns);
  /* L = sum_b c_b Pee_b with Pee = (1 + P_z)/2; by default c_b = dE/N_u (energy-integrated,
   * angle-averaged P_ee of both species) */
  double L = 0.0;
  const double wl = m->dE / (double)m->NU;
  for (int64_t b = 0; b < m->nb; ++b) {
    const double cb = dl_dpee ? dl_dpee[b] : wl;
    L += cb * (0.5 * (1.0 + fin[3 * b + 2]));
    Pb[3 * b + 2] = 0.5 * cb;
  }
  /* derivative tables: d w / d L_a and d B_vac / d theta_v per energy bin */
  adj_tables t;
  t.s2gf = sqrt2gf_km_cm3();
  t.dGe = (double *)malloc(sizeof(double) * m->NE);
  t.dGb = (double *)malloc(sizeof(double) * m->NE);
  t.dGx = (double *)malloc(sizeof(double) * m->NE);
  t.dbx = (double *)malloc(sizeof(double) * m->NE);
  t.dbz = (double *)malloc(sizeof(double) * m->NE);
  const double pref = (m->kappa0 * m->du) * m->dE;
  for (int64_t k = 0; k < m->NE; ++k) {
    const double E = m->E[k];
    t.dGe[k] = pref * ERG_MEV / ((m->p.temp_mev[0] * F3_0) / F2_0) * fermi_dirac(E, m->p.temp_mev[0]);
    t.dGb[k] = pref * ERG_MEV / ((m->p.temp_mev[1] * F3_0) / F2_0) * fermi_dirac(E, m->p.temp_mev[1]);
    t.dGx[k] = -pref * ERG_MEV / ((m->p.temp_mev[2] * F3_0) / F2_0) * fermi_dirac(E, m->p.temp_mev[2]);
    const double om = (VAC_K * m->p.dm2_ev2[0]) / E;
    t.dbx[k] = 4.0 * om * cos(2.0 * m->p.theta[0]);
    t.dbz[k] = 4.0 * om * sin(2.0 * m->p.theta[0]);
  }
  /* reverse pass: each segment is recomputed from its checkpoint, then walked backwards */
  double gth = 0.0, gn0 = 0.0;
  for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
    const int64_t s0 = n0 + sgi * ckpt;
    const int64_t len = (sgi == nseg - 1) ? (N - n0) - sgi * ckpt : ckpt;
    memcpy(m->X, ck + sgi * ns, sizeof(double) * ns);
    m->step = s0;
    for (int64_t i = 0; i < len; ++i) {
      memcpy(tape + i * ns, m->X, sizeof(double) * ns);
      if (i + 1 < len) st |= nbo_step(m, 1);
    }
    for (int64_t i = len - 1; i >= 0; --i)
      reverse_step(m, &t, tape + i * ns, s0 + i, Pb, wbar, &gth, &gn0, Tb, F1b);
  }
  double gLe = 0.0, gLb = 0.0, gLx = 0.0;
  for (int64_t b = 0; b < m->nb; ++b) {
    const int s = (int)(b / (m->NU * m->NE));
    const int64_t k = b % m->NE;
    if (!m->anti[s]) gLe += wbar[b] * t.dGe[k];
    else gLb += wbar[b] * t.dGb[k];
    gLx += wbar[b] * t.dGx[k];
  }
  grad[0] = gLe; grad[1] = gLb; grad[2] = gLx; grad[3] = gth; grad[4] = gn0;
  *loss = L;
  if (state_bar) memcpy(state_bar, Pb, sizeof(double) * ns);
  /* the model is left at the end of the run, as after the forward pass */
  memcpy(m->X, fin, sizeof(double) * ns);
  m->step = N;
  free(ck); free(fin); free(tape); free(Pb); free(Tb); free(F1b); free(wbar);
  free(t.dGe); free(t.dGb); free(t.dGx); free(t.dbx); free(t.dbz);
  return st ? NBO_ENUMERIC : NBO_OK;
}
