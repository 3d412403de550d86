// nb_adjoint.hip -- reverse-mode adjoint of the two-flavour radial integration.
//
// Forward step (state P_n, Bloch vector of one beam; f_i = (h/c_i) B(r_i, J^(i))):
//   Y2 = R(f1/2) P,  Y3 = R(Om) P with Om = f2/2 - (f1 x f2)/8,  Y4 = R(f3) P,
//   Theta = (f1 + 2 f2 + 2 f3 + f4)/6 - (f1 x f4)/12,  P_{n+1} = R(Theta) P / |.|,
// with J^(1) = M(P), J^(2) = M(Y2), J^(3) = M(Y3), J^(4) = M(Y4) the moment sums
// J0 = sum g S y / c, J1 = sum g S y (S = diag(s, 1, s), s = -1 for antineutrinos).
// Its reverse, per step and beam, runs the stages backwards; every moment adjoint is a
// grid-wide sum, so a reverse step has the forward step's four grid barriers:
//   A: renormalisation and final rotation -> Theta-bar -> f4-bar -> sum (J^(4)-bar)
//   B: Y4 broadcast of J^(4)-bar -> f3-bar -> sum (J^(3)-bar)
//   C: Y3 broadcast -> Om-bar -> f2-bar (and part of f1-bar) -> sum (J^(2)-bar)
//   D: Y2 broadcast -> f1-bar -> sum (J^(1)-bar); then the J^(1)-bar broadcast onto P_n.
// For y = R(x) p: p-bar = R(-x) y-bar and x-bar = Jl(x)^T (y x y-bar) with the left
// Jacobian Jl(x) = I + a [x]x + b [x]x^2, a = (1 - cos t)/t^2, b = (t - sin t)/t^3.
// The parameters enter through the weights g (luminosities), B_vac (theta_v) and the
// matter term lambda = sqrt2 G_F n0 (R/r)^p (n0); their adjoints are accumulated per
// thread and summed once at the end.
//
// Memory: the forward pass (nb_adjoint) keeps the state at the start of every segment of
// `ckpt` steps and records all stage moments; a segment is recomputed beam by beam from
// its checkpoint with the recorded moments (no grid synchronisation, the same arithmetic
// as the stepping kernel, hence the same bits) into a tape of `ckpt` states, which the
// reverse steps then read backwards.  Each beam's adjoint state lives in registers of
// the thread that owns it for the whole launch.
#include "nb_device.h"
#include "nb_internal.h"
#include "nb_stage.h"

namespace nb {

// Rotation by the angle vector x (angle |x| about x/|x|, as rotate2) with what its adjoint
// needs: the half-angle quaternion and the left-Jacobian coefficients a, b.
struct Rot {
  double x0, x1, x2;
  double v0, v1, v2, c;  // sin(t/2) x/t, cos(t/2)
  double ja, jb;
};
__device__ __forceinline__ Rot make_rot(double x0, double x1, double x2) {
  Rot r;
  r.x0 = x0;
  r.x1 = x1;
  r.x2 = x2;
  const double t2 = (x0 * x0 + x1 * x1) + x2 * x2;
  const double t = sqrt(t2);
  double s = 0.0, c = 1.0;
  if (t > 0.0) sincos_nb(0.5 * t, s, c);
  const double k = (t > 0.0) ? s / t : 0.0;
  r.v0 = x0 * k;
  r.v1 = x1 * k;
  r.v2 = x2 * k;
  r.c = c;
  if (t < 0.05) {  // series: cancellation-free near zero
    r.ja = (0.5 - t2 / 24.0) + (t2 * t2) / 720.0;
    r.jb = (1.0 / 6.0 - t2 / 120.0) + (t2 * t2) / 5040.0;
  } else {
    r.ja = (2.0 * (s * s)) / t2;
    r.jb = (t - 2.0 * (s * c)) / (t2 * t);
  }
  return r;
}
// y = R(x) p  (quaternion form: t = 2 v x p, y = p + c t + v x t)
__device__ __forceinline__ void rot_fwd(const Rot& r, double p0, double p1, double p2, double& y0,
                                        double& y1, double& y2) {
  double t0 = r.v1 * p2 - r.v2 * p1;
  double t1 = r.v2 * p0 - r.v0 * p2;
  double t2 = r.v0 * p1 - r.v1 * p0;
  t0 = t0 + t0;
  t1 = t1 + t1;
  t2 = t2 + t2;
  y0 = (p0 + r.c * t0) + (r.v1 * t2 - r.v2 * t1);
  y1 = (p1 + r.c * t1) + (r.v2 * t0 - r.v0 * t2);
  y2 = (p2 + r.c * t2) + (r.v0 * t1 - r.v1 * t0);
}
// p-bar += R(-x) y-bar
__device__ __forceinline__ void rot_inv_add(const Rot& r, double y0, double y1, double y2, double* pb) {
  double t0 = r.v2 * y1 - r.v1 * y2;
  double t1 = r.v0 * y2 - r.v2 * y0;
  double t2 = r.v1 * y0 - r.v0 * y1;
  t0 = t0 + t0;
  t1 = t1 + t1;
  t2 = t2 + t2;
  pb[0] += (y0 + r.c * t0) + (r.v2 * t1 - r.v1 * t2);
  pb[1] += (y1 + r.c * t1) + (r.v0 * t2 - r.v2 * t0);
  pb[2] += (y2 + r.c * t2) + (r.v1 * t0 - r.v0 * t1);
}
__device__ __forceinline__ void cross(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
// x-bar = Jl(x)^T w = w - a (x x w) + b x x (x x w)
__device__ __forceinline__ void jl_t(const Rot& r, const double* w, double* o) {
  const double x[3] = {r.x0, r.x1, r.x2};
  double c1[3], c2[3];
  cross(x, w, c1);
  cross(x, c1, c2);
#pragma unroll
  for (int i = 0; i < 3; ++i) o[i] = (w[i] - r.ja * c1[i]) + r.jb * c2[i];
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Deterministic grid sum of NV per-thread values: wave butterflies, the block's waves in
// order, then block 0 adds the block partials in ascending block order within each of its
// thread groups and the group sums in order.  Partials and result travel as tagged words
// (a 32-bit barrier epoch and a 32-bit half of the double), the protocol of the stepping
// kernels' moment reduction: block b publishes its partial as 2 NV words, block 0 polls
// every partial word with all loads in flight and publishes the sums in kFlagCopies copies,
// the other blocks poll the 2 NV words of copy b % kFlagCopies.  The result lands in
// res[0..NV) of every block.  Returns false if the barrier was abandoned (time limit or
// abort).
template <int NV>
__device__ bool grid_sum(const AdjArgs& a, unsigned epoch, double (&v)[NV], double* res,
                         double (*sw)[8], double* sred) {
  constexpr int W = 2 * NV;        // words per partial and per result copy
  constexpr int G = kBlock / W;    // block-0 thread groups
  static_assert(W <= kTagWords64, "tagged slot too small");
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const unsigned want = epoch + 1u;
  const unsigned long long tg = (unsigned long long)want << 32;
  unsigned long long* part = reinterpret_cast<unsigned long long*>(a.sync + kSyncPart);
  unsigned long long* jw = reinterpret_cast<unsigned long long*>(a.sync + kSyncJTag);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double t = wave_sum_f64(v[i]);
    if (lane == 0) sw[wid][i] = t;
  }
  __syncthreads();
  // thread tid < W: half tid % 2 of block sum tid / 2
  unsigned half = 0;
  if (tid < W) {
    double blk = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) blk += sw[w][tid >> 1];
    const unsigned long long bits = as_bits(blk);
    half = (tid & 1) ? (unsigned)(bits >> 32) : (unsigned)bits;
    if (blockIdx.x != 0)
      __hip_atomic_store(part + (size_t)blockIdx.x * kTagWords64 + tid, tg | half, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  if (blockIdx.x != 0) {
    int ok = 1;
    unsigned long long x = 0;
    if (tid < W) {
      const unsigned long long* w = jw + (size_t)(blockIdx.x % kFlagCopies) * kTagWords64 + tid;
      const unsigned long long t0 = wall_clock64();
      for (unsigned it = 1;; ++it) {
        x = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((unsigned)(x >> 32) == want) break;
        if ((it & 31u) == 0u && give_up(a.sync, a.cancel, t0, a.timeout_ticks, it)) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (tid < 64) {
      const unsigned hi = __shfl_down((unsigned)x, 1, 64);
      if (ok && tid < W && (tid & 1) == 0)
        res[tid >> 1] = as_double(((unsigned long long)hi << 32) | (x & 0xffffffffull));
    }
    return !__syncthreads_or(!ok);
  }
  // block 0: thread (g, pos) collects word pos of blocks g, g + G, ... (kFly loads in flight);
  // the even thread of each pair then adds the doubles in ascending block order
  // (few loads in flight: the reverse step keeps many per-beam values live across this call)
  constexpr int kFly = 8;
  int ok = 1;
  const int pos = tid % W, g = tid / W;
  double acc = 0.0;
  const unsigned long long t0 = wall_clock64();
  for (unsigned b0 = g; b0 < gridDim.x; b0 += kFly * G) {
    unsigned long long w[kFly];
    unsigned pend = 0;
    if (g < G) {
#pragma unroll
      for (int i = 0; i < kFly; ++i) {
        const unsigned b = b0 + i * G;
        if (b == 0) w[i] = tg | half;          // block 0's own partial
        else if (b < gridDim.x) pend |= 1u << i;
      }
    }
    for (unsigned it = 1; pend && ok; ++it) {
#pragma unroll
      for (int i = 0; i < kFly; ++i)
        if (pend & (1u << i))
          w[i] = __hip_atomic_load(part + (size_t)(b0 + i * G) * kTagWords64 + pos, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int i = 0; i < kFly; ++i)
        if ((pend & (1u << i)) && (unsigned)(w[i] >> 32) == want) pend &= ~(1u << i);
      if (pend && (it & 31u) == 0u && give_up(a.sync, a.cancel, t0, a.timeout_ticks, it)) ok = 0;
      if (pend && ok) __builtin_amdgcn_s_sleep(1);
    }
    // the two threads of a pair share g, so they run the same iterations of this loop
#pragma unroll
    for (int i = 0; i < kFly; ++i) {
      const unsigned mine = (g < G && b0 + i * G < gridDim.x) ? (unsigned)w[i] : 0u;
      const unsigned hi = __shfl_down(mine, 1, 64);
      if (g < G && (pos & 1) == 0 && b0 + i * G < gridDim.x)
        acc += as_double(((unsigned long long)hi << 32) | mine);
    }
  }
  if (g < G && (pos & 1) == 0) sred[g * NV + (pos >> 1)] = acc;
  if (__syncthreads_or(!ok)) return false;
  if (tid < NV) {
    double tot = 0.0;
    for (int gg = 0; gg < G; ++gg) tot += sred[gg * NV + tid];
    res[tid] = tot;
    const unsigned long long bits = as_bits(tot);
#pragma unroll
    for (int c = 0; c < kFlagCopies; ++c) {
      unsigned long long* q = jw + (size_t)c * kTagWords64 + 2 * tid;
      __hip_atomic_store(q, tg | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(q + 1, tg | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  return true;
}

// Per-beam constants and adjoint registers.
struct AdjBeam {
  double P[3];      // state at the start of the step being reversed
  double Pb[3];     // adjoint of the state
  double F1[3];     // adjoint of f1 (accumulated over phases A, C, D)
  double Tb[3];     // Theta-bar (enters f2-bar and f3-bar)
  double c0, cm, c1, hc0, hcm, hc1;
  double u;
  int s, k;
  bool on;
};

// Adjoint of B at one stage: moment-adjoint contributions S B-bar and c S B-bar of the
// beam, and the direct parameter terms (theta_v through B_vac, n0 through lambda).
__device__ __forceinline__ void b_bar(const AdjArgs& a, const AdjBeam& q, const double* Bb, double c,
                                      const Radial& g, double (&red)[6], double (&gacc)[5]) {
  const double sg = q.s ? -1.0 : 1.0;
  const double S0 = sg * Bb[0], S1 = Bb[1], S2 = sg * Bb[2];
  red[0] += S0;
  red[1] += S1;
  red[2] += S2;
  red[3] += c * S0;
  red[4] += c * S1;
  red[5] += c * S2;
  const double* dbx = a.dtab + 3 * (size_t)a.NE;
  const double* dbz = a.dtab + 4 * (size_t)a.NE;
  gacc[3] += Bb[0] * dbx[q.k] + Bb[2] * dbz[q.k];
  gacc[4] += sg * Bb[2] * (a.s2gf * g.qp);
}

// Broadcast of a moment adjoint (J0-bar | J1-bar) onto a stage state y at cos c:
// y-bar = g S (J0-bar/c + J1-bar); the weight adjoint (S y).(J0-bar/c + J1-bar) feeds the
// luminosity gradients.
__device__ __forceinline__ void m_bar(const AdjArgs& a, const AdjBeam& q, const double* Jb, double c,
                                      const double* y, double* yb, double (&gacc)[5]) {
  const double sg = q.s ? -1.0 : 1.0;
  const double v0 = Jb[0] / c + Jb[3], v1 = Jb[1] / c + Jb[4], v2 = Jb[2] / c + Jb[5];
  const double w = a.tab[(size_t)(2 + q.s) * a.NE + q.k];
  yb[0] = w * (sg * v0);
  yb[1] = w * v1;
  yb[2] = w * (sg * v2);
  const double wb = ((sg * y[0]) * v0 + y[1] * v1) + (sg * y[2]) * v2;
  gacc[q.s] += wb * a.dtab[(size_t)q.s * a.NE + q.k];
  gacc[2] += wb * a.dtab[2 * (size_t)a.NE + q.k];
}

__device__ __forceinline__ void stage_f(const AdjArgs& a, const AdjBeam& q, const double* J, const Radial& g,
                                        double c, double hc, double* f) {
  double nn[3];
  nunu<3>(J, g.mu, c, nn);
  gen2(q.s, a.tab[q.k], a.tab[a.NE + q.k], g.lam, nn, hc, f);
}

// Beam b's fixed labels, its adjoint initialised from the cotangent (L = sum_b c_b Pee_b,
// Pee = (1 + P_z)/2).
__device__ __forceinline__ void beam_init(const AdjArgs& a, long long b, bool on, AdjBeam& q) {
  q.on = on;
  const long long bb = on ? b : 0;
  const long long row = bb / a.NE;
  q.k = (int)(bb - row * a.NE);
  q.s = (int)(row / a.NU);
  q.u = u_of((int)(row - (long long)q.s * a.NU), a.NU);
  const double cb = on ? (a.cot ? a.cot[b] : a.cot_const) : 0.0;
  q.Pb[0] = 0.0;
  q.Pb[1] = 0.0;
  q.Pb[2] = 0.5 * cb;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    q.F1[c] = 0.0;
    q.Tb[c] = 0.0;
    q.P[c] = 0.0;
  }
  q.c0 = q.cm = q.c1 = 1.0;
  q.hc0 = q.hcm = q.hc1 = 0.0;
}

// Recompute beam b's states over a segment of len steps from its checkpoint with the
// recorded moments (the stepping kernel's arithmetic, hence its bits) into the tape.
__device__ __forceinline__ void recompute_segment(const AdjArgs& a, const AdjBeam& q, long long b, long long seg,
                                                  long long s0, long long len) {
  const long long plane = a.plane;
  const double* ck = a.ck + (size_t)seg * 3 * plane;
  double P0 = ck[b], P1 = ck[b + plane], P2 = ck[b + 2 * plane];
  for (long long t = 0; t < len; ++t) {
    double* tp = a.tape + (size_t)t * 3 * plane;
    tp[b] = P0;
    tp[b + plane] = P1;
    tp[b + 2 * plane] = P2;
    if (t + 1 == len) break;
    const long long n = s0 + t;
    const double r0 = a.rs + (double)n * a.h;
    const double rm = r0 + 0.5 * a.h;
    const double r1 = a.rs + (double)(n + 1) * a.h;
    const Radial g0 = radial(a.R, a.ne_power, a.lam0, r0), gm = radial(a.R, a.ne_power, a.lam0, rm),
                 g1 = radial(a.R, a.ne_power, a.lam0, r1);
    const RowGeo rg = row_geo(q.u, a.h, g0, gm, g1);
    const double* J = a.Jhist + (size_t)n * 24;
    double n1[3], n2[3], n3[3], n4[3], f1[3], f2[3], f3[3], f4[3];
    nunu<3>(J, g0.mu, rg.c0, n1);
    nunu<3>(J + 6, gm.mu, rg.cm, n2);
    nunu<3>(J + 12, gm.mu, rg.cm, n3);
    nunu<3>(J + 18, g1.mu, rg.c1, n4);
    const double bx = a.tab[q.k], bz = a.tab[a.NE + q.k];
    gen2(q.s, bx, bz, g0.lam, n1, rg.hc0, f1);
    gen2(q.s, bx, bz, gm.lam, n2, rg.hcm, f2);
    gen2(q.s, bx, bz, gm.lam, n3, rg.hcm, f3);
    gen2(q.s, bx, bz, g1.lam, n4, rg.hc1, f4);
    const double cr0 = f1[1] * f4[2] - f1[2] * f4[1];
    const double cr1 = f1[2] * f4[0] - f1[0] * f4[2];
    const double cr2 = f1[0] * f4[1] - f1[1] * f4[0];
    const double t0 = (((f1[0] + 2.0 * f2[0]) + 2.0 * f3[0]) + f4[0]) * (1.0 / 6.0) - cr0 * (1.0 / 12.0);
    const double t1 = (((f1[1] + 2.0 * f2[1]) + 2.0 * f3[1]) + f4[1]) * (1.0 / 6.0) - cr1 * (1.0 / 12.0);
    const double t2 = (((f1[2] + 2.0 * f2[2]) + 2.0 * f3[2]) + f4[2]) * (1.0 / 6.0) - cr2 * (1.0 / 12.0);
    rotate2(t0, t1, t2, P0, P1, P2);
    if (a.renorm) {   // as the forward stepper: one Newton step for 1/sqrt from 1
      const double nrm2 = (P0 * P0 + P1 * P1) + P2 * P2;
      const double inv = fma(-0.5, nrm2, 1.5);
      P0 = P0 * inv;
      P1 = P1 * inv;
      P2 = P2 * inv;
    }
  }
}

// The state at the start of the step being reversed (tape slot t) and the beam's geometry
// at the step's three stage radii.
__device__ __forceinline__ void load_step(const AdjArgs& a, AdjBeam& B, long long b, long long t,
                                          const Radial& g0, const Radial& gm, const Radial& g1) {
  const double* tp = a.tape + (size_t)t * 3 * a.plane;
  B.P[0] = tp[b];
  B.P[1] = tp[b + a.plane];
  B.P[2] = tp[b + 2 * a.plane];
  const RowGeo rg = row_geo(B.u, a.h, g0, gm, g1);
  B.c0 = rg.c0; B.cm = rg.cm; B.c1 = rg.c1;
  B.hc0 = rg.hc0; B.hcm = rg.hcm; B.hc1 = rg.hc1;
}

// A: P_{n+1} = R(Theta) P_n / |.|  ->  Theta-bar, f4-bar
__device__ __forceinline__ void phase_a(const AdjArgs& a, AdjBeam& B, const double (*sJ)[6], const Radial& g0,
                                        const Radial& gm, const Radial& g1, double (&red)[6], double (&gacc)[5]) {
  double f1[3], f2[3], f3[3], f4[3], cr[3];
  stage_f(a, B, sJ[0], g0, B.c0, B.hc0, f1);
  stage_f(a, B, sJ[1], gm, B.cm, B.hcm, f2);
  stage_f(a, B, sJ[2], gm, B.cm, B.hcm, f3);
  stage_f(a, B, sJ[3], g1, B.c1, B.hc1, f4);
  cross(f1, f4, cr);
  double th[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    th[c] = (((f1[c] + 2.0 * f2[c]) + 2.0 * f3[c]) + f4[c]) * (1.0 / 6.0) - cr[c] * (1.0 / 12.0);
  const Rot R = make_rot(th[0], th[1], th[2]);
  double Pp[3];
  rot_fwd(R, B.P[0], B.P[1], B.P[2], Pp[0], Pp[1], Pp[2]);
  double Ppb[3] = {B.Pb[0], B.Pb[1], B.Pb[2]};
  if (a.renorm) {
    // y = P (1.5 - |P|^2 / 2): P-bar = (1.5 - |P|^2 / 2) y-bar - P (P . y-bar)
    const double sf = fma(-0.5, (Pp[0] * Pp[0] + Pp[1] * Pp[1]) + Pp[2] * Pp[2], 1.5);
    const double d = (Pp[0] * Ppb[0] + Pp[1] * Ppb[1]) + Pp[2] * Ppb[2];
    Ppb[0] = sf * Ppb[0] - Pp[0] * d;
    Ppb[1] = sf * Ppb[1] - Pp[1] * d;
    Ppb[2] = sf * Ppb[2] - Pp[2] * d;
  }
  B.Pb[0] = B.Pb[1] = B.Pb[2] = 0.0;
  rot_inv_add(R, Ppb[0], Ppb[1], Ppb[2], B.Pb);
  double om[3], tb[3], c4[3], c1v[3], f4b[3];
  cross(Pp, Ppb, om);
  jl_t(R, om, tb);
  cross(f4, tb, c4);
  cross(tb, f1, c1v);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    B.F1[c] = tb[c] / 6.0 - c4[c] / 12.0;
    f4b[c] = tb[c] / 6.0 - c1v[c] / 12.0;
    B.Tb[c] = tb[c];
  }
  const double Bb[3] = {B.hc1 * f4b[0], B.hc1 * f4b[1], B.hc1 * f4b[2]};
  b_bar(a, B, Bb, B.c1, g1, red, gacc);
}
// B: Y4 = R(f3) P  ->  f3-bar
__device__ __forceinline__ void phase_b(const AdjArgs& a, AdjBeam& B, const double (*sJ)[6], const double* Jb,
                                        const Radial& gm, double (&red)[6], double (&gacc)[5]) {
  double f3[3], Y[3], Yb[3], om[3], f3b[3];
  stage_f(a, B, sJ[2], gm, B.cm, B.hcm, f3);
  const Rot R = make_rot(f3[0], f3[1], f3[2]);
  rot_fwd(R, B.P[0], B.P[1], B.P[2], Y[0], Y[1], Y[2]);
  m_bar(a, B, Jb, B.c1, Y, Yb, gacc);
  rot_inv_add(R, Yb[0], Yb[1], Yb[2], B.Pb);
  cross(Y, Yb, om);
  jl_t(R, om, f3b);
#pragma unroll
  for (int c = 0; c < 3; ++c) f3b[c] += B.Tb[c] / 3.0;
  const double Bb[3] = {B.hcm * f3b[0], B.hcm * f3b[1], B.hcm * f3b[2]};
  b_bar(a, B, Bb, B.cm, gm, red, gacc);
}
// C: Y3 = R(Om) P, Om = f2/2 - (f1 x f2)/8  ->  f2-bar, f1-bar
__device__ __forceinline__ void phase_c(const AdjArgs& a, AdjBeam& B, const double (*sJ)[6], const double* Jb,
                                        const Radial& g0, const Radial& gm, double (&red)[6], double (&gacc)[5]) {
  double f1[3], f2[3], cr[3], Y[3], Yb[3], om[3], ob[3], a1[3], a2[3], f2b[3];
  stage_f(a, B, sJ[0], g0, B.c0, B.hc0, f1);
  stage_f(a, B, sJ[1], gm, B.cm, B.hcm, f2);
  cross(f1, f2, cr);
  const Rot R = make_rot(0.5 * f2[0] - 0.125 * cr[0], 0.5 * f2[1] - 0.125 * cr[1],
                         0.5 * f2[2] - 0.125 * cr[2]);
  rot_fwd(R, B.P[0], B.P[1], B.P[2], Y[0], Y[1], Y[2]);
  m_bar(a, B, Jb, B.cm, Y, Yb, gacc);
  rot_inv_add(R, Yb[0], Yb[1], Yb[2], B.Pb);
  cross(Y, Yb, om);
  jl_t(R, om, ob);
  cross(ob, f1, a1);
  cross(f2, ob, a2);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    f2b[c] = (0.5 * ob[c] - a1[c] / 8.0) + B.Tb[c] / 3.0;
    B.F1[c] -= a2[c] / 8.0;
  }
  const double Bb[3] = {B.hcm * f2b[0], B.hcm * f2b[1], B.hcm * f2b[2]};
  b_bar(a, B, Bb, B.cm, gm, red, gacc);
}
// D: Y2 = R(f1/2) P  ->  f1-bar complete
__device__ __forceinline__ void phase_d(const AdjArgs& a, AdjBeam& B, const double (*sJ)[6], const double* Jb,
                                        const Radial& g0, double (&red)[6], double (&gacc)[5]) {
  double f1[3], Y[3], Yb[3], om[3], ob[3];
  stage_f(a, B, sJ[0], g0, B.c0, B.hc0, f1);
  const Rot R = make_rot(0.5 * f1[0], 0.5 * f1[1], 0.5 * f1[2]);
  rot_fwd(R, B.P[0], B.P[1], B.P[2], Y[0], Y[1], Y[2]);
  m_bar(a, B, Jb, B.cm, Y, Yb, gacc);
  rot_inv_add(R, Yb[0], Yb[1], Yb[2], B.Pb);
  cross(Y, Yb, om);
  jl_t(R, om, ob);
#pragma unroll
  for (int c = 0; c < 3; ++c) B.F1[c] += 0.5 * ob[c];
  const double Bb[3] = {B.hc0 * B.F1[0], B.hc0 * B.F1[1], B.hc0 * B.F1[2]};
  b_bar(a, B, Bb, B.c0, g0, red, gacc);
}
// J^(1) = M(P_n): the moment adjoint broadcast onto the state itself
__device__ __forceinline__ void phase_e(const AdjArgs& a, AdjBeam& B, const double* Jb, double (&gacc)[5]) {
  double Yb[3];
  m_bar(a, B, Jb, B.c0, B.P, Yb, gacc);
  B.Pb[0] += Yb[0];
  B.Pb[1] += Yb[1];
  B.Pb[2] += Yb[2];
}

// Adjoint registers of beam b kept in the workspace between phases (spill mode): P-bar,
// f1-bar, Theta-bar as nine planes of a.plane doubles.
__device__ __forceinline__ void adj_load(const AdjArgs& a, AdjBeam& B, long long b) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    B.Pb[c] = a.spill[(size_t)c * a.plane + b];
    B.F1[c] = a.spill[(size_t)(3 + c) * a.plane + b];
    B.Tb[c] = a.spill[(size_t)(6 + c) * a.plane + b];
  }
}
__device__ __forceinline__ void adj_store(const AdjArgs& a, const AdjBeam& B, long long b) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a.spill[(size_t)c * a.plane + b] = B.Pb[c];
    a.spill[(size_t)(3 + c) * a.plane + b] = B.F1[c];
    a.spill[(size_t)(6 + c) * a.plane + b] = B.Tb[c];
  }
}

// BPT > 0: thread gt owns beams gt + i nthr (i < BPT) and keeps their adjoint registers for
// the whole launch.  BPT = 0 (spill mode, any number of beams): each phase loops over the
// thread's beams gt, gt + nthr, ..., reading and writing their adjoint registers in the
// workspace and recomputing the state and geometry from the tape.
template <int BPT>
__global__ void __launch_bounds__(kBlock) k_adjoint2(AdjArgs a) {
  __shared__ double sJ[4][6];
  __shared__ double sRes[8];
  __shared__ double sw[kBlock / 64][8];
  __shared__ double sred[kBlock];
  constexpr int NQ = BPT > 0 ? BPT : 1;
  if (launch_aborted(a.sync)) return;
  const int tid = threadIdx.x;
  const long long nthr = (long long)gridDim.x * kBlock;
  const long long gt = (long long)blockIdx.x * kBlock + tid;
  AdjBeam q[NQ];
  if constexpr (BPT > 0) {
#pragma unroll
    for (int i = 0; i < BPT; ++i) beam_init(a, gt + i * nthr, gt + i * nthr < a.nb, q[i]);
  } else {
    for (long long b = gt; b < a.nb; b += nthr) {
      beam_init(a, b, true, q[0]);
      adj_store(a, q[0], b);
    }
  }
  // every beam of this thread (register mode: its BPT slots; spill mode: all of them, each
  // loaded and stored around fn)
  auto each = [&](auto fn, bool with_state, long long t, const Radial& g0, const Radial& gm, const Radial& g1) {
    if constexpr (BPT > 0) {
#pragma unroll
      for (int i = 0; i < BPT; ++i)
        if (q[i].on) fn(q[i], gt + i * nthr);
    } else {
      for (long long b = gt; b < a.nb; b += nthr) {
        beam_init(a, b, true, q[0]);
        adj_load(a, q[0], b);
        if (with_state) load_step(a, q[0], b, t, g0, gm, g1);
        fn(q[0], b);
        adj_store(a, q[0], b);
      }
    }
  };
  double gacc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  unsigned epoch = 0;
  bool ok = true;
  for (long long seg = a.nseg - 1; ok && seg >= 0; --seg) {
    const long long s0 = a.n0 + seg * a.ckpt;
    const long long len = min(a.ckpt, a.n0 + a.nsteps - s0);
    // -- recompute the segment's states from its checkpoint with the recorded moments
    if constexpr (BPT > 0) {
#pragma unroll
      for (int i = 0; i < BPT; ++i)
        if (q[i].on) recompute_segment(a, q[i], gt + i * nthr, seg, s0, len);
    } else {
      for (long long b = gt; b < a.nb; b += nthr) {
        beam_init(a, b, true, q[0]);
        recompute_segment(a, q[0], b, seg, s0, len);
      }
    }
    // -- reverse steps of the segment
    for (long long t = len - 1; ok && t >= 0; --t) {
      const long long n = s0 + t;
      const double r0 = a.rs + (double)n * a.h;
      const double rm = r0 + 0.5 * a.h;
      const double r1 = a.rs + (double)(n + 1) * a.h;
      const Radial g0 = radial(a.R, a.ne_power, a.lam0, r0), gm = radial(a.R, a.ne_power, a.lam0, rm),
                   g1 = radial(a.R, a.ne_power, a.lam0, r1);
      if (tid < 24) sJ[tid / 6][tid % 6] = a.Jhist[(size_t)n * 24 + tid];
      __syncthreads();
      double red[6];
      double Jb[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) red[c] = 0.0;
      each([&](AdjBeam& B, long long b) {
        if constexpr (BPT > 0) load_step(a, B, b, t, g0, gm, g1);
        phase_a(a, B, sJ, g0, gm, g1, red, gacc);
      }, true, t, g0, gm, g1);
      if (!(ok = grid_sum<6>(a, epoch++, red, sRes, sw, sred))) break;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Jb[c] = g1.mu * sRes[c];
        Jb[3 + c] = -(g1.mu * sRes[3 + c]);
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) red[c] = 0.0;
      each([&](AdjBeam& B, long long) { phase_b(a, B, sJ, Jb, gm, red, gacc); }, true, t, g0, gm, g1);
      if (!(ok = grid_sum<6>(a, epoch++, red, sRes, sw, sred))) break;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Jb[c] = gm.mu * sRes[c];
        Jb[3 + c] = -(gm.mu * sRes[3 + c]);
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) red[c] = 0.0;
      each([&](AdjBeam& B, long long) { phase_c(a, B, sJ, Jb, g0, gm, red, gacc); }, true, t, g0, gm, g1);
      if (!(ok = grid_sum<6>(a, epoch++, red, sRes, sw, sred))) break;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Jb[c] = gm.mu * sRes[c];
        Jb[3 + c] = -(gm.mu * sRes[3 + c]);
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) red[c] = 0.0;
      each([&](AdjBeam& B, long long) { phase_d(a, B, sJ, Jb, g0, red, gacc); }, true, t, g0, gm, g1);
      if (!(ok = grid_sum<6>(a, epoch++, red, sRes, sw, sred))) break;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Jb[c] = g0.mu * sRes[c];
        Jb[3 + c] = -(g0.mu * sRes[3 + c]);
      }
      each([&](AdjBeam& B, long long) { phase_e(a, B, Jb, gacc); }, true, t, g0, gm, g1);
    }
  }
  if (!ok) return;
  if (a.state_bar) {
    if constexpr (BPT > 0) {
#pragma unroll
      for (int i = 0; i < BPT; ++i) {
        if (!q[i].on) continue;
        const long long b = gt + i * nthr;
        a.state_bar[b] = q[i].Pb[0];
        a.state_bar[b + a.nb] = q[i].Pb[1];
        a.state_bar[b + 2 * a.nb] = q[i].Pb[2];
      }
    } else {
      for (long long b = gt; b < a.nb; b += nthr)
#pragma unroll
        for (int c = 0; c < 3; ++c) a.state_bar[b + c * a.nb] = a.spill[(size_t)c * a.plane + b];
    }
  }
  if (grid_sum<5>(a, epoch++, gacc, sRes, sw, sred) && blockIdx.x == 0 && tid < 5) a.out[tid] = sRes[tid];
}

template __global__ void k_adjoint2<0>(AdjArgs);
template __global__ void k_adjoint2<1>(AdjArgs);
template __global__ void k_adjoint2<2>(AdjArgs);
template __global__ void k_adjoint2<4>(AdjArgs);

}  // namespace nb
