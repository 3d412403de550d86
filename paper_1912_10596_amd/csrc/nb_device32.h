// nb_device32.h -- single-precision per-beam arithmetic of the mixed-precision stepper.
//
// The exact 3x3 exponential exp(-iK) psi of nb_device.h carried out in FP32 for the
// NB_FP32_STATE mode (the generators come from FP64 row constants in the caller).  There
// is no bit-for-bit contract here: divisions use the hardware reciprocal, sin/cos a short
// polynomial after a three-part reduction, and the moment sums and the renormalisation
// stay in FP64 in the caller.  Accuracy is that of FP32 per step;
// rotation angles must stay well below 2^15 (pi/2 multiples) for the reduction to hold.
#pragma once
#include <hip/hip_runtime.h>

// No bit-for-bit contract binds this arithmetic, so products and sums may fuse into fma
// (the rest of the library is compiled without contraction).
#pragma clang fp contract(fast)

namespace nb {

// sin and cos in FP32: x = k pi/2 + r (three-part split of pi/2 applied with fma),
// Taylor polynomials of degree 9 (sin) and 10 (cos) on |r| <= pi/4.
__device__ __forceinline__ void sincos_f(float x, float& sn, float& cs) {
  // k = x 2/pi rounded to the nearest integer by adding 1.5 2^23 (|x| < 2^21); the low bits
  // of t are k mod 4
  const float t = fmaf(x, 0x1.45f306p-1f, 0x1.8p23f);
  const float k = t - 0x1.8p23f;
  float r = fmaf(-k, 0x1.92p+0f, x);
  r = fmaf(-k, 0x1.fb6p-12f, r);
  r = fmaf(-k, -0x1.777a5cp-25f, r);
  const float r2 = r * r;
  float ps = 1.0f / 362880.0f;
  ps = fmaf(ps, r2, -1.0f / 5040.0f);
  ps = fmaf(ps, r2, 1.0f / 120.0f);
  ps = fmaf(ps, r2, -1.0f / 6.0f);
  const float s = fmaf(r2 * r, ps, r);
  float pc = -1.0f / 3628800.0f;
  pc = fmaf(pc, r2, 1.0f / 40320.0f);
  pc = fmaf(pc, r2, -1.0f / 720.0f);
  pc = fmaf(pc, r2, 1.0f / 24.0f);
  pc = fmaf(pc, r2, -0.5f);
  const float c = fmaf(r2, pc, 1.0f);
  const int q = __float_as_int(t) & 3;
  sn = (q == 0) ? s : ((q == 1) ? c : ((q == 2) ? -s : -c));
  cs = (q == 0) ? c : ((q == 1) ? -s : ((q == 2) ? -c : s));
}
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }
// cos x - 1 and sin(x)/x from x2 = x^2 for x^2 <= 4, without range reduction: Taylor series
// to x^16 / 16! and x^14 / 15! (remainders below 4e-9 at |x| = 2); cos x - 1 is accurate
// relative to its own size.
__device__ __forceinline__ void cosm1_sinc_f(float x2, float& cm1, float& snc) {
  float pc = 1.0f / 20922789888000.0f;
  pc = fmaf(pc, x2, -1.0f / 87178291200.0f);
  pc = fmaf(pc, x2, 1.0f / 479001600.0f);
  pc = fmaf(pc, x2, -1.0f / 3628800.0f);
  pc = fmaf(pc, x2, 1.0f / 40320.0f);
  pc = fmaf(pc, x2, -1.0f / 720.0f);
  pc = fmaf(pc, x2, 1.0f / 24.0f);
  pc = fmaf(pc, x2, -0.5f);
  cm1 = x2 * pc;
  float ps = -1.0f / 1307674368000.0f;
  ps = fmaf(ps, x2, 1.0f / 6227020800.0f);
  ps = fmaf(ps, x2, -1.0f / 39916800.0f);
  ps = fmaf(ps, x2, 1.0f / 362880.0f);
  ps = fmaf(ps, x2, -1.0f / 5040.0f);
  ps = fmaf(ps, x2, 1.0f / 120.0f);
  ps = fmaf(ps, x2, -1.0f / 6.0f);
  snc = fmaf(ps, x2, 1.0f);
}

struct cplxf {
  float re, im;
};
__device__ __forceinline__ cplxf mkf(float re, float im) { return cplxf{re, im}; }
__device__ __forceinline__ cplxf cmulf(cplxf a, cplxf b) {
  return mkf(fmaf(a.re, b.re, -(a.im * b.im)), fmaf(a.re, b.im, a.im * b.re));
}
__device__ __forceinline__ cplxf rmulf(float a, cplxf b) { return mkf(a * b.re, a * b.im); }
__device__ __forceinline__ cplxf conjf_(cplxf a) { return mkf(a.re, -a.im); }
__device__ __forceinline__ float norm2f(cplxf a) { return fmaf(a.re, a.re, a.im * a.im); }

struct Herm3f {
  float d0, d1, d2;
  cplxf o01, o02, o12;
};
// The sums below are written as single fma chains (one product rounded on its own, the
// rest fused), which halves the instruction count against separate products and adds.
__device__ __forceinline__ float cnorm2vf(const cplxf v[3]) {
  return fmaf(v[0].re, v[0].re, fmaf(v[0].im, v[0].im, fmaf(v[1].re, v[1].re, fmaf(v[1].im, v[1].im,
              fmaf(v[2].re, v[2].re, v[2].im * v[2].im)))));
}
// u^+ v
__device__ __forceinline__ cplxf dotcf(const cplxf u[3], const cplxf v[3]) {
  return mkf(fmaf(u[0].re, v[0].re, fmaf(u[0].im, v[0].im, fmaf(u[1].re, v[1].re, fmaf(u[1].im, v[1].im,
                 fmaf(u[2].re, v[2].re, u[2].im * v[2].im))))),
             fmaf(u[0].re, v[0].im, fmaf(-u[0].im, v[0].re, fmaf(u[1].re, v[1].im, fmaf(-u[1].im, v[1].re,
                 fmaf(u[2].re, v[2].im, -(u[2].im * v[2].re)))))));
}
// (K0 - hm) v: rows (d0, x, y), (x^*, d1, z), (y^*, z^*, d2)
__device__ __forceinline__ void k0_minusf(const cplxf v[3], float d0, float d1, float d2, cplxf x,
                                          cplxf y, cplxf z, cplxf o[3]) {
  o[0] = mkf(fmaf(d0, v[0].re, fmaf(x.re, v[1].re, fmaf(-x.im, v[1].im, fmaf(y.re, v[2].re, -(y.im * v[2].im))))),
             fmaf(d0, v[0].im, fmaf(x.re, v[1].im, fmaf(x.im, v[1].re, fmaf(y.re, v[2].im, y.im * v[2].re)))));
  o[1] = mkf(fmaf(x.re, v[0].re, fmaf(x.im, v[0].im, fmaf(d1, v[1].re, fmaf(z.re, v[2].re, -(z.im * v[2].im))))),
             fmaf(x.re, v[0].im, fmaf(-x.im, v[0].re, fmaf(d1, v[1].im, fmaf(z.re, v[2].im, z.im * v[2].re)))));
  o[2] = mkf(fmaf(y.re, v[0].re, fmaf(y.im, v[0].im, fmaf(z.re, v[1].re, fmaf(z.im, v[1].im, d2 * v[2].re)))),
             fmaf(y.re, v[0].im, fmaf(-y.im, v[0].re, fmaf(z.re, v[1].im, fmaf(-z.im, v[1].re, d2 * v[2].im)))));
}

// Eigen-split of exp(-i K) in FP32, the algorithm of the FP64 version (largest eigenvalue
// by Halley steps on the characteristic cubic, its eigenvector from the column of
// adj(K0 - l1) with the largest diagonal entry, the plane angle from P psi), except that
// v1 is normalised with the hardware rsqrt (FP32 cannot hold |K0|^5): psi = al v1 + pp with
// pp orthogonal to v1, kp = (K0 - hm) pp, and the phases phi (of v1) and th (of the
// orthogonal plane), so that
//   exp(-i K) psi = e^{-i phi} al v1 + cos(th) pp - i sin(th)/th kp   (global phase dropped).
// Returns false if K is zero (exp(-iK) psi = psi up to a phase).  The caller evaluates the
// phases without range reduction when |phi| and th are at most 2 (the resolved steps this
// mode runs, where every generator's eigenvalues stay near or below one).
struct Split3f {
  cplxf v1[3], pp[3], kp[3], al;
  float phi, th2;   // th2 = th^2
};
__device__ __forceinline__ bool split3_f(const Herm3f& K, const cplxf psi[3], Split3f& o) {
  const float tr = ((K.d0 + K.d1) + K.d2) * (1.0f / 3.0f);
  const float a0 = K.d0 - tr, a1 = K.d1 - tr, a2 = K.d2 - tr;
  const cplxf x = K.o01, y = K.o02, z = K.o12;
  const float nx = norm2f(x), ny = norm2f(y), nz = norm2f(z);
  const float s2 = fmaf(a0, a0, fmaf(a1, a1, a2 * a2));
  const float p = fmaf(0.5f, s2, (nx + ny) + nz);
  const cplxf xz = cmulf(x, z);
  const float t = fmaf(xz.re, y.re, xz.im * y.im);
  const float q = fmaf(a0, fmaf(a1, a2, -nz), fmaf(-a1, ny, fmaf(-a2, nx, 2.0f * t)));
  if (!(p > 0.0f)) return false;
  const float sg = (q < 0.0f) ? -1.0f : 1.0f;
  const float qa = sg * q;
  // start: 0.9 times 2 sqrt(p/3), the square root by halving the exponent in the bit
  // pattern (at most 6.1 % above it).  The root lies between sqrt(p) and 2 sqrt(p/3), so the
  // start is within 10 % of it on either side, from where two Halley steps leave a relative
  // error below 1e-8 (worst case over the cubic's shapes and the estimate's range).
  float lam = 1.8f * __int_as_float((int)(((unsigned)__float_as_int(p * (1.0f / 3.0f)) >> 1) + 0x1FC00000u));
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float l2 = lam * lam;
    const float fv = fmaf(lam, l2 - p, -qa);
    const float dv = fmaf(3.0f, l2, -p);
    const float den = fmaf(dv, dv, -((3.0f * lam) * fv));
    lam = lam - (fv * dv) * rcp_f(den);
  }
  const float l1 = sg * lam;
  const float p0 = a0 - l1, p1 = a1 - l1, p2 = a2 - l1;
  const float c00 = fmaf(p1, p2, -nz), c11 = fmaf(p0, p2, -ny), c22 = fmaf(p0, p1, -nx);
  const cplxf u = mkf(fmaf(y.re, z.re, fmaf(y.im, z.im, -(p2 * x.re))), fmaf(y.im, z.re, fmaf(-y.re, z.im, -(p2 * x.im))));
  const cplxf v = mkf(fmaf(x.re, z.re, fmaf(-x.im, z.im, -(p1 * y.re))), fmaf(x.re, z.im, fmaf(x.im, z.re, -(p1 * y.im))));
  const cplxf tt = mkf(fmaf(x.re, y.re, fmaf(x.im, y.im, -(p0 * z.re))), fmaf(x.re, y.im, fmaf(-x.im, y.re, -(p0 * z.im))));
  int jc = 0;
  float cjj = c00;
  if (c11 > cjj) { jc = 1; cjj = c11; }
  if (c22 > cjj) { jc = 2; cjj = c22; }
  cplxf best[3];
  best[0] = (jc == 0) ? mkf(c00, 0.0f) : ((jc == 1) ? u : v);
  best[1] = (jc == 0) ? conjf_(u) : ((jc == 1) ? mkf(c11, 0.0f) : tt);
  best[2] = (jc == 0) ? conjf_(v) : ((jc == 1) ? conjf_(tt) : mkf(c22, 0.0f));
  const float nb = cnorm2vf(best);
  if (!(nb > 0.0f)) return false;
  const float inb = rsqrtf(nb);
#pragma unroll
  for (int c = 0; c < 3; ++c) o.v1[c] = rmulf(inb, best[c]);
  const float hm = -0.5f * l1;
  const float d0 = a0 - hm, d1 = a1 - hm, d2 = a2 - hm;
  o.al = dotcf(o.v1, psi);
#pragma unroll
  for (int c = 0; c < 3; ++c)   // psi - al v1
    o.pp[c] = mkf(fmaf(-o.al.re, o.v1[c].re, fmaf(o.al.im, o.v1[c].im, psi[c].re)),
                  fmaf(-o.al.re, o.v1[c].im, fmaf(-o.al.im, o.v1[c].re, psi[c].im)));
  k0_minusf(o.pp, d0, d1, d2, x, y, z, o.kp);
  // (K0 - hm)^2 = th^2 on the plane: th^2 = |kp|^2 / |pp|^2 (0 for pp = 0)
  const float npp = cnorm2vf(o.pp);
  o.th2 = (npp > 0.0f) ? cnorm2vf(o.kp) * rcp_f(npp) : 0.0f;
  o.phi = l1 - hm;
  return true;
}

// cos and sin of phi, cos th and sin(th)/th: Taylor series in phi^2 and th^2 when both
// are at most 4, else range reduction.
__device__ __forceinline__ void phases_f(const Split3f& e, float& cp, float& sp, float& ct, float& sc) {
  const float p2 = e.phi * e.phi;
  if (p2 <= 4.0f && e.th2 <= 4.0f) {
    float cm1, snc;
    cosm1_sinc_f(p2, cm1, snc);
    cp = 1.0f + cm1;
    sp = e.phi * snc;
    cosm1_sinc_f(e.th2, cm1, sc);
    ct = 1.0f + cm1;
  } else {
    const float th = sqrtf(e.th2);
    float st;
    sincos_f(e.phi, sp, cp);
    sincos_f(th, st, ct);
    sc = (th > 0.0f) ? st * rcp_f(th) : 1.0f;
  }
}
// psi <- exp(-i K) psi (up to a global phase) in FP32.
__device__ __forceinline__ void exp3_apply_f(const Herm3f& K, cplxf psi[3]) {
  Split3f e;
  if (!split3_f(K, psi, e)) return;
  float sp, cp, ct, sc;
  phases_f(e, cp, sp, ct, sc);
  const cplxf ap = cmulf(e.al, mkf(cp, -sp));
#pragma unroll
  for (int c = 0; c < 3; ++c)   // ap v1 + cos(th) pp - i sin(th)/th kp
    psi[c] = mkf(fmaf(ap.re, e.v1[c].re, fmaf(-ap.im, e.v1[c].im, fmaf(ct, e.pp[c].re, sc * e.kp[c].im))),
                 fmaf(ap.re, e.v1[c].im, fmaf(ap.im, e.v1[c].re, fmaf(ct, e.pp[c].im, -(sc * e.kp[c].re)))));
}

// The increment d = exp(-i K) psi - psi in FP32 (global phase of exp dropped as above),
// formed without cancellation: cos x - 1 = -2 sin^2(x/2), sin x = 2 sin(x/2) cos(x/2), so
//   d = ((cos phi - 1) - i sin phi) al v1 + (cos th - 1) pp - i sin(th)/th kp
// is accurate relative to its own size, and psi + d is formed by the caller in FP64.
__device__ __forceinline__ void exp3_incr_f(const Herm3f& K, const cplxf psi[3], cplxf d[3]) {
  Split3f e;
  if (!split3_f(K, psi, e)) {
    d[0] = d[1] = d[2] = mkf(0.0f, 0.0f);
    return;
  }
  float cpm1, sp, ctm1, sc;
  const float p2 = e.phi * e.phi;
  if (p2 <= 4.0f && e.th2 <= 4.0f) {
    float snc;
    cosm1_sinc_f(p2, cpm1, snc);
    sp = e.phi * snc;
    cosm1_sinc_f(e.th2, ctm1, sc);
  } else {
    const float th = sqrtf(e.th2);
    float sh, ch, tsh, tch;
    sincos_f(0.5f * e.phi, sh, ch);
    sincos_f(0.5f * th, tsh, tch);
    cpm1 = -2.0f * (sh * sh);
    sp = 2.0f * (sh * ch);
    ctm1 = -2.0f * (tsh * tsh);
    sc = (th > 0.0f) ? (2.0f * (tsh * tch)) * rcp_f(th) : 1.0f;
  }
  const cplxf ap = cmulf(e.al, mkf(cpm1, -sp));
#pragma unroll
  for (int c = 0; c < 3; ++c)
    d[c] = mkf(fmaf(ap.re, e.v1[c].re, fmaf(-ap.im, e.v1[c].im, fmaf(ctm1, e.pp[c].re, sc * e.kp[c].im))),
               fmaf(ap.re, e.v1[c].im, fmaf(ap.im, e.v1[c].re, fmaf(ctm1, e.pp[c].im, -(sc * e.kp[c].re)))));
}

}  // namespace nb

#pragma clang fp contract(off)
