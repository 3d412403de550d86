// nb_device32.h -- single-precision per-beam arithmetic of the mixed-precision stepper.
//
// The same operations as the FP64 primitives of nb_device.h (stage generator, the exact
// 3x3 exponential exp(-iK) psi, the commutator i[A,B]) carried out in FP32 for the
// NB_FP32_STATE mode.  There is no bit-for-bit contract here: divisions use the hardware
// reciprocal, sin/cos a short polynomial after a three-part reduction, and the moment sums
// and the renormalisation stay in FP64 in the caller.  Accuracy is that of FP32 per step;
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
  const float k = rintf(x * 0x1.45f306p-1f);
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
  const int q = ((int)k) & 3;
  sn = (q == 0) ? s : ((q == 1) ? c : ((q == 2) ? -s : -c));
  cs = (q == 0) ? c : ((q == 1) ? -s : ((q == 2) ? -c : s));
}
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

struct cplxf {
  float re, im;
};
__device__ __forceinline__ cplxf mkf(float re, float im) { return cplxf{re, im}; }
__device__ __forceinline__ cplxf cmulf(cplxf a, cplxf b) {
  return mkf(fmaf(a.re, b.re, -(a.im * b.im)), fmaf(a.re, b.im, a.im * b.re));
}
__device__ __forceinline__ cplxf cmulf_conja(cplxf a, cplxf b) {  // conj(a) * b
  return mkf(fmaf(a.re, b.re, a.im * b.im), fmaf(a.re, b.im, -(a.im * b.re)));
}
__device__ __forceinline__ cplxf cmulf_conjb(cplxf a, cplxf b) {  // a * conj(b)
  return mkf(fmaf(a.re, b.re, a.im * b.im), fmaf(a.im, b.re, -(a.re * b.im)));
}
__device__ __forceinline__ cplxf rmulf(float a, cplxf b) { return mkf(a * b.re, a * b.im); }
__device__ __forceinline__ cplxf caddf(cplxf a, cplxf b) { return mkf(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cplxf csubf(cplxf a, cplxf b) { return mkf(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cplxf conjf_(cplxf a) { return mkf(a.re, -a.im); }
__device__ __forceinline__ float norm2f(cplxf a) { return fmaf(a.re, a.re, a.im * a.im); }

struct Herm3f {
  float d0, d1, d2;
  cplxf o01, o02, o12;
};
__device__ __forceinline__ cplxf hatf(const Herm3f& h, int a, int b) {
  if (a == b) return mkf(a == 0 ? h.d0 : (a == 1 ? h.d1 : h.d2), 0.0f);
  const cplxf o = (a + b == 1) ? h.o01 : ((a + b == 2) ? h.o02 : h.o12);
  return a < b ? o : conjf_(o);
}
__device__ __forceinline__ Herm3f hscalef(float s, const Herm3f& h) {
  return Herm3f{s * h.d0, s * h.d1, s * h.d2, rmulf(s, h.o01), rmulf(s, h.o02), rmulf(s, h.o12)};
}
__device__ __forceinline__ void haxpyf(Herm3f& acc, float a, const Herm3f& K) {
  acc.d0 = fmaf(a, K.d0, acc.d0);
  acc.d1 = fmaf(a, K.d1, acc.d1);
  acc.d2 = fmaf(a, K.d2, acc.d2);
  acc.o01 = mkf(fmaf(a, K.o01.re, acc.o01.re), fmaf(a, K.o01.im, acc.o01.im));
  acc.o02 = mkf(fmaf(a, K.o02.re, acc.o02.re), fmaf(a, K.o02.im, acc.o02.im));
  acc.o12 = mkf(fmaf(a, K.o12.re, acc.o12.re), fmaf(a, K.o12.im, acc.o12.im));
}
// C(A,B) = i [A,B]
__device__ __forceinline__ Herm3f icommf(const Herm3f& A, const Herm3f& B) {
  cplxf X[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      X[a][b] = caddf(caddf(cmulf(hatf(A, a, 0), hatf(B, 0, b)), cmulf(hatf(A, a, 1), hatf(B, 1, b))),
                      cmulf(hatf(A, a, 2), hatf(B, 2, b)));
  Herm3f C;
  C.d0 = -2.0f * X[0][0].im;
  C.d1 = -2.0f * X[1][1].im;
  C.d2 = -2.0f * X[2][2].im;
  C.o01 = mkf(-(X[0][1].im + X[1][0].im), X[0][1].re - X[1][0].re);
  C.o02 = mkf(-(X[0][2].im + X[2][0].im), X[0][2].re - X[2][0].re);
  C.o12 = mkf(-(X[1][2].im + X[2][1].im), X[1][2].re - X[2][1].re);
  return C;
}

__device__ __forceinline__ void cross3cf(const cplxf u[3], const cplxf v[3], cplxf o[3]) {
  o[0] = csubf(cmulf(u[1], v[2]), cmulf(u[2], v[1]));
  o[1] = csubf(cmulf(u[2], v[0]), cmulf(u[0], v[2]));
  o[2] = csubf(cmulf(u[0], v[1]), cmulf(u[1], v[0]));
}
__device__ __forceinline__ float cnorm2vf(const cplxf v[3]) {
  return (norm2f(v[0]) + norm2f(v[1])) + norm2f(v[2]);
}
__device__ __forceinline__ void k0_minusf(const cplxf v[3], float d0, float d1, float d2, cplxf x,
                                          cplxf y, cplxf z, cplxf o[3]) {
  o[0] = caddf(caddf(rmulf(d0, v[0]), cmulf(x, v[1])), cmulf(y, v[2]));
  o[1] = caddf(caddf(cmulf_conja(x, v[0]), rmulf(d1, v[1])), cmulf(z, v[2]));
  o[2] = caddf(caddf(cmulf_conja(y, v[0]), cmulf_conja(z, v[1])), rmulf(d2, v[2]));
}

// Eigen-split of exp(-i K) in FP32, the algorithm of the FP64 version (largest eigenvalue
// by Newton on the characteristic cubic, its eigenvector from the largest row cross
// product): psi = al v1 + pp with pp orthogonal to v1, kp = (K0 - hm) pp, and the phases
// phi (of v1) and th (of the orthogonal plane), so that
//   exp(-i K) psi = e^{-i phi} al v1 + cos(th) pp - i sin(th)/th kp   (global phase dropped).
// Returns false if K is zero (exp(-iK) psi = psi up to a phase).
struct Split3f {
  cplxf v1[3], pp[3], kp[3], al;
  float phi, th;
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
  float lam = 2.0f * sqrtf(p * (1.0f / 3.0f));
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    const float l2 = lam * lam;
    const float fv = fmaf(lam, l2 - p, -qa);
    const float dv = fmaf(3.0f, l2, -p);
    lam = lam - fv * rcp_f(dv);
  }
  const float l1 = sg * lam;
  const cplxf r0[3] = {mkf(a0 - l1, 0.0f), x, y};
  const cplxf r1[3] = {conjf_(x), mkf(a1 - l1, 0.0f), z};
  const cplxf r2[3] = {conjf_(y), conjf_(z), mkf(a2 - l1, 0.0f)};
  cplxf best[3];
  float nb;
  {
    cplxf c[3];
    cross3cf(r0, r1, c);
    nb = cnorm2vf(c);
    best[0] = c[0]; best[1] = c[1]; best[2] = c[2];
  }
  {
    cplxf c[3];
    cross3cf(r0, r2, c);
    const float n = cnorm2vf(c);
    if (n > nb) {
      best[0] = c[0]; best[1] = c[1]; best[2] = c[2];
      nb = n;
    }
  }
  {
    cplxf c[3];
    cross3cf(r1, r2, c);
    const float n = cnorm2vf(c);
    if (n > nb) {
      best[0] = c[0]; best[1] = c[1]; best[2] = c[2];
      nb = n;
    }
  }
  if (!(nb > 0.0f)) return false;
  const float inb = rsqrtf(nb);
#pragma unroll
  for (int c = 0; c < 3; ++c) o.v1[c] = rmulf(inb, best[c]);
  const float hm = -0.5f * l1;
  const float d0 = a0 - hm, d1 = a1 - hm, d2 = a2 - hm;
  {
    const float nc0 = norm2f(o.v1[0]), nc1 = norm2f(o.v1[1]), nc2 = norm2f(o.v1[2]);
    int m = 0;
    float ncm = nc0;
    if (nc1 < ncm) { m = 1; ncm = nc1; }
    if (nc2 < ncm) { m = 2; ncm = nc2; }
    const cplxf vm = (m == 0) ? o.v1[0] : ((m == 1) ? o.v1[1] : o.v1[2]);
    cplxf w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplxf tm = cmulf_conjb(o.v1[c], vm);
      w[c] = (c == m) ? mkf(1.0f - ncm, 0.0f) : mkf(-tm.re, -tm.im);
    }
    const float inw = rsqrtf(cnorm2vf(w));
    const cplxf u[3] = {rmulf(inw, w[0]), rmulf(inw, w[1]), rmulf(inw, w[2])};
    cplxf ku[3];
    k0_minusf(u, d0, d1, d2, x, y, z, ku);
    o.th = sqrtf(cnorm2vf(ku));
  }
  o.al = caddf(caddf(cmulf_conja(o.v1[0], psi[0]), cmulf_conja(o.v1[1], psi[1])),
               cmulf_conja(o.v1[2], psi[2]));
#pragma unroll
  for (int c = 0; c < 3; ++c) o.pp[c] = csubf(psi[c], cmulf(o.al, o.v1[c]));
  k0_minusf(o.pp, d0, d1, d2, x, y, z, o.kp);
  o.phi = l1 - hm;
  return true;
}

// psi <- exp(-i K) psi (up to a global phase) in FP32.
__device__ __forceinline__ void exp3_apply_f(const Herm3f& K, cplxf psi[3]) {
  Split3f e;
  if (!split3_f(K, psi, e)) return;
  float sp, cp, st, ct;
  sincos_f(e.phi, sp, cp);
  sincos_f(e.th, st, ct);
  const float sc = (e.th > 0.0f) ? st * rcp_f(e.th) : 1.0f;
  const cplxf ap = cmulf(e.al, mkf(cp, -sp));
#pragma unroll
  for (int c = 0; c < 3; ++c)
    psi[c] = caddf(cmulf(ap, e.v1[c]),
                   mkf(fmaf(ct, e.pp[c].re, sc * e.kp[c].im), fmaf(ct, e.pp[c].im, -(sc * e.kp[c].re))));
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
  float sh, ch, tsh, tch;
  sincos_f(0.5f * e.phi, sh, ch);
  sincos_f(0.5f * e.th, tsh, tch);
  const float cpm1 = -2.0f * (sh * sh), sp = 2.0f * (sh * ch);
  const float ctm1 = -2.0f * (tsh * tsh);
  const float sc = (e.th > 0.0f) ? (2.0f * (tsh * tch)) * rcp_f(e.th) : 1.0f;
  const cplxf ap = cmulf(e.al, mkf(cpm1, -sp));
#pragma unroll
  for (int c = 0; c < 3; ++c)
    d[c] = caddf(cmulf(ap, e.v1[c]),
                 mkf(fmaf(ctm1, e.pp[c].re, sc * e.kp[c].im), fmaf(ctm1, e.pp[c].im, -(sc * e.kp[c].re))));
}

}  // namespace nb

#pragma clang fp contract(off)
