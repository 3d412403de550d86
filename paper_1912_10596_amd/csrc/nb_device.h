// nb_device.h -- CDNA4 device primitives of the bulb-model stepper.
//
// Arithmetic specification (bit-for-bit contract with the CPU reference): every
// multiply and add below is rounded separately (the library is compiled with
// -ffp-contract=off); fma appears only where written; division and sqrt are the IEEE
// correctly rounded operations; sin/cos are the library's own (Cody-Waite reduction by
// pi/2 in three parts, Taylor polynomials of degree 17/18); moment sums are exact
// integer sums of fixed-point values (rounded to nearest), so their result does not depend on the
// grid shape or on the order in which waves and blocks finish.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

constexpr double kTwo56 = 72057594037927936.0;
constexpr double kTwo62 = 4611686018427387904.0;
constexpr double kTwo64 = 18446744073709551616.0;

// ------------------------------------------------------------------ sin / cos
// sin and cos of one argument.  Reduction x = k pi/2 + r with k the nearest integer to 2x/pi and a
// three-part split of pi/2 (each part applied with one fma); then Taylor series of sin
// (to r^17) and cos (to r^18) by Horner in r^2; the quadrant k mod 4 picks signs.
__device__ __forceinline__ void sincos_nb(double x, double& sn, double& cs) {
  // k = the exact product x 2/pi rounded once to the nearest integer: the fma adds
  // 1.5 2^52 and rounds in a binade of unit spacing, so t - 1.5 2^52 = k and the low bits
  // of t are k mod 4 (|x| < 2^50)
  const double t = fma(x, 0x1.45f306dc9c883p-1, 0x1.8p52);
  const double k = t - 0x1.8p52;
  double r = fma(-k, 0x1.921fb54442d18p+0, x);
  r = fma(-k, 0x1.1a62633145c07p-54, r);
  r = fma(-k, -0x1.f1976b7ed8fbcp-110, r);
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
  const int quad = (int)(__double_as_longlong(t) & 3);
  const double a = (quad & 1) ? c : s;    // |sin| candidate
  const double b = (quad & 1) ? s : c;    // |cos| candidate
  sn = (quad & 2) ? -a : a;
  cs = ((quad + 1) & 2) ? -b : b;
}

// The same sin/cos with its constants read from a table (for instance in LDS, so that a
// kernel short of registers does not hold them in VGPRs): c = the values sincos_coefs writes.
constexpr int kSinCosTab = 21;
__device__ __forceinline__ void sincos_coefs(double* c) {
  c[0] = 0x1.45f306dc9c883p-1; c[1] = 0x1.921fb54442d18p+0; c[2] = 0x1.1a62633145c07p-54;
  c[3] = -0x1.f1976b7ed8fbcp-110;
  c[4] = 1.0 / 355687428096000.0; c[5] = -1.0 / 1307674368000.0; c[6] = 1.0 / 6227020800.0;
  c[7] = -1.0 / 39916800.0; c[8] = 1.0 / 362880.0; c[9] = -1.0 / 5040.0; c[10] = 1.0 / 120.0;
  c[11] = -1.0 / 6.0;
  c[12] = -1.0 / 6402373705728000.0; c[13] = 1.0 / 20922789888000.0; c[14] = -1.0 / 87178291200.0;
  c[15] = 1.0 / 479001600.0; c[16] = -1.0 / 3628800.0; c[17] = 1.0 / 40320.0; c[18] = -1.0 / 720.0;
  c[19] = 1.0 / 24.0; c[20] = -0.5;
}
__device__ __forceinline__ void sincos_tab(double x, const double* c, double& sn, double& cs) {
  const double t = fma(x, c[0], 0x1.8p52);
  const double k = t - 0x1.8p52;
  double r = fma(-k, c[1], x);
  r = fma(-k, c[2], r);
  r = fma(-k, c[3], r);
  const double r2 = r * r;
  double ps = c[4];
#pragma unroll
  for (int i = 5; i <= 11; ++i) ps = fma(ps, r2, c[i]);
  const double s = fma(r2 * r, ps, r);
  double pc = c[12];
#pragma unroll
  for (int i = 13; i <= 20; ++i) pc = fma(pc, r2, c[i]);
  const double cc = fma(r2, pc, 1.0);
  const int quad = (int)(__double_as_longlong(t) & 3);
  const double a = (quad & 1) ? cc : s;
  const double b = (quad & 1) ? s : cc;
  sn = (quad & 2) ? -a : a;
  cs = ((quad + 1) & 2) ? -b : b;
}

// ------------------------------------------------------------- fixed point
// 128-bit two's complement integer held as two 64-bit halves.
struct I128 {
  unsigned long long lo;
  long long hi;
};
__device__ __forceinline__ I128 i128_zero() { return I128{0ull, 0ll}; }
__device__ __forceinline__ I128 i128_from(long long v) {
  return I128{(unsigned long long)v, v >> 63};
}
__device__ __forceinline__ I128 i128_add(I128 a, I128 b) {
  I128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (long long)(r.lo < a.lo);
  return r;
}
// Sign-magnitude conversion: |x| = hi 2^64 + lo, (double)hi * 2^64 + (double)lo.
__device__ __forceinline__ double i128_to_double(I128 x) {
  const bool neg = x.hi < 0;
  unsigned long long lo = x.lo, hi = (unsigned long long)x.hi;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (unsigned long long)(lo == 0ull);
  }
  const double v = (double)hi * kTwo64 + (double)lo;
  return neg ? -v : v;
}
// trunc(v * scale) as an integer; flags values outside (-limit, limit) (NaN included).
// Used for the per-angle J0 terms (limit 2^62).
// Status bits a lane reports (the kernels OR them into the status word at the end of a
// launch): 1 = a moment contribution left its fixed-point range (or a state norm reached 2,
// NaN included); 8 = a renormalisation met |psi|^2 (|P|^2) further from 1 than the
// rounding of a unitary step can explain: kRenormTol for FP64 states, kRenormTol32 for
// FP32-stored states (their own rounding is ~6e-8).
constexpr double kRenormTol = 1e-8;
constexpr double kRenormTol32 = 1e-5;
__device__ __forceinline__ long long to_fix(double v, double scale, double limit, int& err) {
  const double x = v * scale;
  if (!(fabs(x) < limit)) {
    err |= 1;
    return 0;
  }
  return (long long)x;
}
// A beam's moment contribution: the exact product v * ws (ws = weight * 2^e1) rounded
// once to the nearest integer, ties to even.  The fma adds 1.5 2^52 and rounds in a binade
// of unit spacing, so the integer sits in the low mantissa bits: the result's bit pattern
// is kFixMagic + that integer (exact for |v ws| <= 2^51, which the caller's per-beam state
// check guarantees).  Callers add bit patterns and take kFixMagic off once per count of
// contributions; all of it is modulo 2^64, so the true sum comes out exactly.
constexpr unsigned long long kFixMagic = 0x4338000000000000ull;
__device__ __forceinline__ unsigned long long fix_bits(double v, double ws) {
  return (unsigned long long)__double_as_longlong(fma(v, ws, 0x1.8p52));
}
// Butterfly sum over the 64 lanes of a wavefront; every lane gets the total.
__device__ __forceinline__ I128 wave_sum(I128 a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    I128 o;
    o.lo = __shfl_xor(a.lo, off, 64);
    o.hi = __shfl_xor(a.hi, off, 64);
    a = i128_add(a, o);
  }
  return a;
}

// ------------------------------------------------------------------ complex
struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx mk(double re, double im) { return cplx{re, im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return mk(fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re));
}
__device__ __forceinline__ cplx cmul_conjb(cplx a, cplx b) {  // a * conj(b)
  return mk(fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -(a.re * b.im)));
}
__device__ __forceinline__ cplx cmul_conja(cplx a, cplx b) {  // conj(a) * b
  return mk(fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re)));
}
__device__ __forceinline__ cplx rmul(double a, cplx b) { return mk(a * b.re, a * b.im); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return mk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return mk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cplx conjg(cplx a) { return mk(a.re, -a.im); }
__device__ __forceinline__ double norm2(cplx a) { return fma(a.re, a.re, a.im * a.im); }

// Hermitian 3x3: real diagonal d0..d2, upper entries o01, o02, o12.
struct Herm3 {
  double d0, d1, d2;
  cplx o01, o02, o12;
};

// a0 b0 + a1 b1 + a2 b2 (complex): the six real products accumulated with fma from the
// last one up (the specification's fused three-term complex dot product).
__device__ __forceinline__ cplx dot3_mul(cplx a0, cplx b0, cplx a1, cplx b1, cplx a2, cplx b2) {
  return mk(fma(a0.re, b0.re, fma(-a0.im, b0.im, fma(a1.re, b1.re, fma(-a1.im, b1.im,
                fma(a2.re, b2.re, -(a2.im * b2.im)))))),
            fma(a0.re, b0.im, fma(a0.im, b0.re, fma(a1.re, b1.im, fma(a1.im, b1.re,
                fma(a2.re, b2.im, a2.im * b2.re))))));
}

__device__ __forceinline__ cplx dotc(const cplx u[3], const cplx v[3]) {  // u^+ v
  return dot3_mul(conjg(u[0]), v[0], conjg(u[1]), v[1], conjg(u[2]), v[2]);
}
// |v0|^2 + |v1|^2 + |v2|^2, fused from the last square up
__device__ __forceinline__ double cnorm2v(const cplx v[3]) {
  return fma(v[0].re, v[0].re, fma(v[0].im, v[0].im, fma(v[1].re, v[1].re, fma(v[1].im, v[1].im,
             fma(v[2].re, v[2].re, v[2].im * v[2].im)))));
}

// psi <- exp(-i K) psi up to a global phase (three flavours).  K0 = traceless part of K,
// l1 its eigenvalue of largest magnitude (3 Halley steps on the characteristic cubic
// l^3 - p l - q from a start within 23 % above it: full FP64 accuracy), c a
// column of adj(K0 - l1) (its eigenvector, v1 = c / |c|).  On the plane orthogonal to v1,
// K0 - hm with hm = -l1/2 squares to th^2, so the plane is propagated by the closed-form
// 2x2 exponential of Eq. U:
//   psi' = e^{-i (l1 - hm)} (v1^+ psi) v1 + cos(th) P psi - i sin(th)/th (K0 - hm) P psi,
// P = I - v1 v1^+, th = |(K0 - hm) w| / |w| for any w in the plane, here w = P psi.
// Nothing is normalised: (v1^+ psi) v1 = al c with al = (c^+ psi) / |c|^2.  The magnitudes
// then grow like |K0|^5; with the sin/cos reduction (phases below 2^50) the form holds for
// 2^-100 < |K0| < 1e15; |K0|^2 / 2 <= 2^-200 is taken as K0 = 0 (error below 1e-30).
// (K0 - hm) v: rows (d0, x, y), (x^*, d1, z), (y^*, z^*, d2), each a complex dot product
// with the real diagonal entry, fused from the last product up
__device__ __forceinline__ void k0_minus(const cplx v[3], double d0, double d1, double d2,
                                         cplx x, cplx y, cplx z, cplx o[3]) {
  o[0] = mk(fma(d0, v[0].re, fma(x.re, v[1].re, fma(-x.im, v[1].im, fma(y.re, v[2].re, -(y.im * v[2].im))))),
            fma(d0, v[0].im, fma(x.re, v[1].im, fma(x.im, v[1].re, fma(y.re, v[2].im, y.im * v[2].re)))));
  o[1] = mk(fma(x.re, v[0].re, fma(x.im, v[0].im, fma(d1, v[1].re, fma(z.re, v[2].re, -(z.im * v[2].im))))),
            fma(x.re, v[0].im, fma(-x.im, v[0].re, fma(d1, v[1].im, fma(z.re, v[2].im, z.im * v[2].re)))));
  o[2] = mk(fma(y.re, v[0].re, fma(y.im, v[0].im, fma(z.re, v[1].re, fma(z.im, v[1].im, d2 * v[2].re)))),
            fma(y.re, v[0].im, fma(-y.im, v[0].re, fma(z.re, v[1].im, fma(-z.im, v[1].re, d2 * v[2].im)))));
}

__device__ __forceinline__ void exp3_apply(const Herm3& K, cplx psi[3]) {
  const double tr = ((K.d0 + K.d1) + K.d2) * (1.0 / 3.0);
  const double a0 = K.d0 - tr, a1 = K.d1 - tr, a2 = K.d2 - tr;
  const cplx x = K.o01, y = K.o02, z = K.o12;
  const double nx = norm2(x), ny = norm2(y), nz = norm2(z);
  const double s2 = fma(a0, a0, fma(a1, a1, a2 * a2));
  const double p = fma(0.5, s2, (nx + ny) + nz);
  const cplx xz = cmul(x, z);
  const double t = fma(xz.re, y.re, xz.im * y.im);
  const double q = fma(a0, fma(a1, a2, -nz), fma(-a1, ny, fma(-a2, nx, 2.0 * t)));
  if (!(p > 0x1p-200)) return;
  const double sg = (q < 0.0) ? -1.0 : 1.0;
  const double qa = sg * q;
  // start: 2 sqrt(p/3) by halving the exponent in the bit pattern of p/3 (at most 6.1 %
  // above the square root, never below: above the root and within 23 % of it)
  double lam = 2.0 * __longlong_as_double(
                         (long long)(((unsigned long long)__double_as_longlong(p * (1.0 / 3.0)) >> 1) +
                                     0x1FF8000000000000ull));
#pragma unroll
  for (int it = 0; it < 3; ++it) {   // Halley: l - f f' / (f'^2 - f f''/2), f'' = 6 l
    const double l2 = lam * lam;
    const double fv = fma(lam, l2 - p, -qa);
    const double dv = fma(3.0, l2, -p);
    const double den = fma(dv, dv, -((3.0 * lam) * fv));
    lam = lam - (fv * dv) / den;
  }
  const double l1 = sg * lam;
  // eigenvector c: the column of adj(K0 - l1) = mu v1 v1^+ (mu > 0) with the largest
  // diagonal entry (first wins ties).  p_i = a_i - l1; diagonal cofactors p1 p2 - |z|^2,
  // p0 p2 - |y|^2, p0 p1 - |x|^2; above the diagonal u = y z^* - p2 x, v = x z - p1 y,
  // t = x^* y - p0 z; columns (c00, u^*, v^*), (u, c11, t^*), (v, t, c22).
  const double p0 = a0 - l1, p1 = a1 - l1, p2 = a2 - l1;
  const double c00 = fma(p1, p2, -nz), c11 = fma(p0, p2, -ny), c22 = fma(p0, p1, -nx);
  const cplx u = mk(fma(y.re, z.re, fma(y.im, z.im, -(p2 * x.re))),
                    fma(y.im, z.re, fma(-y.re, z.im, -(p2 * x.im))));
  const cplx v = mk(fma(x.re, z.re, fma(-x.im, z.im, -(p1 * y.re))),
                    fma(x.re, z.im, fma(x.im, z.re, -(p1 * y.im))));
  const cplx tt = mk(fma(x.re, y.re, fma(x.im, y.im, -(p0 * z.re))),
                     fma(x.re, y.im, fma(-x.im, y.re, -(p0 * z.im))));
  int jc = 0;
  double cjj = c00;
  if (c11 > cjj) { jc = 1; cjj = c11; }
  if (c22 > cjj) { jc = 2; cjj = c22; }
  cplx best[3];
  best[0] = (jc == 0) ? mk(c00, 0.0) : ((jc == 1) ? u : v);
  best[1] = (jc == 0) ? conjg(u) : ((jc == 1) ? mk(c11, 0.0) : tt);
  best[2] = (jc == 0) ? conjg(v) : ((jc == 1) ? conjg(tt) : mk(c22, 0.0));
  const double nb = cnorm2v(best);
  if (!(nb > 0.0)) return;
  const double hm = -0.5 * l1;
  const double d0 = a0 - hm, d1 = a1 - hm, d2 = a2 - hm;
  const cplx al = rmul(1.0 / nb, dotc(best, psi));   // (v1^+ psi) v1 = al c
  cplx pp[3], kp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)   // P psi = psi - al c
    pp[c] = mk(fma(-al.re, best[c].re, fma(al.im, best[c].im, psi[c].re)),
               fma(-al.re, best[c].im, fma(-al.im, best[c].re, psi[c].im)));
  k0_minus(pp, d0, d1, d2, x, y, z, kp);
  // (K0 - hm)^2 = th^2 on the plane: th = |(K0 - hm) P psi| / |P psi| (0 for P psi = 0)
  const double npp = cnorm2v(pp);
  const double th = (npp > 0.0) ? sqrt(cnorm2v(kp) / npp) : 0.0;
  const double phi = l1 - hm;
  double sp, cp, st, ct;
  sincos_nb(phi, sp, cp);
  sincos_nb(th, st, ct);
  const double sc = (th > 0.0) ? st / th : 1.0;
  const cplx ap = cmul(al, mk(cp, -sp));
#pragma unroll
  for (int c = 0; c < 3; ++c)   // ap c + cos(th) P psi - i sin(th)/th (K0 - hm) P psi
    psi[c] = mk(fma(ap.re, best[c].re, fma(-ap.im, best[c].im, fma(ct, pp[c].re, sc * kp[c].im))),
                fma(ap.re, best[c].im, fma(ap.im, best[c].re, fma(ct, pp[c].im, -(sc * kp[c].re)))));
}

// Bloch-vector rotation about x by |x| (two flavours): unit quaternion
// (cos|x|/2, sin(|x|/2) x/|x|), P' = P + w t + v x t with t = 2 v x P.  TAB: the sin/cos
// constants are read from tab (sincos_coefs) instead of immediates.
template <bool TAB = false>
__device__ __forceinline__ void rotate2(const double x0, const double x1, const double x2,
                                        double& P0, double& P1, double& P2,
                                        const double* tab = nullptr) {
  const double t2 = (x0 * x0 + x1 * x1) + x2 * x2;
  const double th = sqrt(t2);
  if (th == 0.0) return;
  double s, c;
  if constexpr (TAB) sincos_tab(0.5 * th, tab, s, c);
  else sincos_nb(0.5 * th, s, c);
  const double k = s / th;
  const double v0 = x0 * k, v1 = x1 * k, v2 = x2 * k;
  double t0 = v1 * P2 - v2 * P1;
  double t1 = v2 * P0 - v0 * P2;
  double tt = v0 * P1 - v1 * P0;
  t0 = t0 + t0;
  t1 = t1 + t1;
  tt = tt + tt;
  const double u0 = v1 * tt - v2 * t1;
  const double u1 = v2 * t0 - v0 * tt;
  const double u2 = v0 * t1 - v1 * t0;
  P0 = (P0 + c * t0) + u0;
  P1 = (P1 + c * t1) + u1;
  P2 = (P2 + c * tt) + u2;
}

}  // namespace nb
