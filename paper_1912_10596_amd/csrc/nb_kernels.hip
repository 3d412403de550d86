// nb_kernels.hip -- persistent CDNA4 kernels of the bulb-model radial stepper.
//
// One persistent launch advances every beam by `nsteps` radial steps.  Work unit: one
// (species, emission-bin) row of N_E beams per wavefront -- the paper's NBeam with its
// SIMD loop over energy bins (Sec. 3.3) mapped onto 64 lanes.  Per RK stage each wave
//   1. streams its rows' state planes (SoA, coalesced 64 x 8 B per load),
//   2. rebuilds every beam's stage generator from the global stage moments (no per-beam
//      stage storage: F_1..F_{i-1} are recomputed from J^(1..i-1)),
//   3. applies the exact exponential to get the stage state Y_i (Eq. U),
//   4. accumulates the beam's moment contribution as a 64-bit fixed-point integer; the
//      row's energy sum is a wavefront butterfly of 128-bit integers, then the angle sum
//      (1/cos weighting for J0) is added to per-lane totals,
// then the block folds its waves through LDS, publishes its partial as epoch-tagged words,
// and every block gathers all partials into J^(i) (no release flag; agent-scope atomics).
// Four barriers per step; the final pass writes rho_{n+1} and also produces the next
// step's stage-1 moments.
#include "nb_device.h"
#include "nb_device32.h"
#include "nb_internal.h"
#include "nb_stage.h"
#include <type_traits>

namespace nb {

__device__ __forceinline__ Radial radial_at(const StepArgs& a, double r) {
  return radial(a.R, a.ne_power, a.lam0, r);
}

// Grid-wide reduction of the stage moments with tagged words, gathered by every block.
// Every 64-bit word that crosses blocks carries the epoch of the barrier it belongs to, so
// a reader knows from the word itself whether it is current, and no arrival or release
// word (and no store acknowledgement before one) lies on the critical path:
//  * every block publishes its partial (NV 128-bit sums, each below 2^95 in magnitude) as
//    2 NV words of a 16-bit tag and a 48-bit chunk: bits 0..47, then bits 48..95, into its
//    slot of the region of the epoch's parity;
//  * every block polls all partial words (each of its threads owns one chunk position of
//    a set of blocks and re-polls only the words not yet current, all loads in flight),
//    adds the chunks in 64-bit integers (below 2^61 for up to kMaxBlocks blocks) and
//    combines them to the exact 128-bit totals: the same integers in every block, whatever
//    the order, so every block holds the same moments after one publish-and-poll hop.
// The two parity regions make every word safe to rewrite: block b writes its slot of
// parity e % 2 at epoch e only after reading every partial of epoch e - 1, and every
// block c wrote that partial only after it had finished reading epoch e - 2, the previous
// contents of the same parity region.  All words are zeroed before each launch and
// epochs start at 1, so a tag equal to the wanted epoch is never stale (the 16-bit tags
// repeat only every 65536 barriers).
// Returns false if the barrier was abandoned (time limit or abort).
constexpr unsigned long long kMask48 = (1ull << 48) - 1ull;
// 48-bit chunk k of a 128-bit value below 2^95 in magnitude: k = 0 the unsigned bits
// 0..47, k = 1 the signed bits 48..95 (as a 48-bit field of the tagged word, and as its
// integer value).
__device__ __forceinline__ unsigned long long chunk_field(const I128& x, int k) {
  return (k ? ((x.lo >> 48) | ((unsigned long long)x.hi << 16)) : x.lo) & kMask48;
}
__device__ __forceinline__ long long chunk_value(unsigned long long field, int k) {
  return k ? ((long long)(field << 16) >> 16) : (long long)field;
}

// blk: the block's partial (threads tid < NV hold component tid); own: unused (every
// block reads its own partial back with the others).  MAXE adds one more word to every
// partial, efield (thread NV): the block's largest error estimate as the top 48 bits of its
// binary form (a non-negative double, so the integer order of the fields is the order of
// the values); every block takes the largest field, which lands in *sE.
// NM moment groups of NV / NM components: J0 | J1 (| J_sc | J_ss); J1 is at scale 2^e1,
// the others at 2^e0.
// BS: threads per block (the launch's block size), so that the thread groups and every
// poll address are compile-time constants.
template <int NV, bool MAXE, int NM, int BS>
__device__ __forceinline__ bool grid_reduce(const StepArgs& a, unsigned epoch, I128 blk, long long own,
                            unsigned long long efield, double* sJ, long long* sacc, double* sE) {
  constexpr int W = 2 * NV + (MAXE ? 1 : 0);   // words per partial
  constexpr int G = BS / W;                    // thread groups, one chunk position per thread
  static_assert(W <= kTagWords64, "tagged slot too small");
  const int tid = threadIdx.x;
  const unsigned want = epoch + 1u;
  const unsigned long long tag16 = (unsigned long long)(want & 0xffffu);
  unsigned long long* part = reinterpret_cast<unsigned long long*>(a.sync + kSyncPart) +
                             (size_t)(epoch & 1u) * kMaxBlocks * kTagWords64;
  unsigned long long* slot = part + (size_t)blockIdx.x * kTagWords64;
  if (tid < NV) {
    __hip_atomic_store(slot + 2 * tid, (tag16 << 48) | chunk_field(blk, 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(slot + 2 * tid + 1, (tag16 << 48) | chunk_field(blk, 1), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  if (MAXE && tid == NV)
    __hip_atomic_store(slot + 2 * NV, (tag16 << 48) | efield, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int ok = 1;
  const int pos = tid % W, g = tid / W;
  long long acc = 0;
  if (g < G) {
    const unsigned long long t0 = wall_clock64();
    for (unsigned b0 = g; b0 < gridDim.x && ok; b0 += 16 * G) {
      unsigned pend = 0;
      unsigned long long w[16];
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (b0 + i * G < gridDim.x) pend |= 1u << i;
      for (unsigned it = 1; pend; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (pend & (1u << i))
            w[i] = __hip_atomic_load(part + (size_t)(b0 + i * G) * kTagWords64 + pos, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if ((pend & (1u << i)) && (w[i] >> 48) == tag16) {
            if (MAXE && pos == 2 * NV) acc = max(acc, (long long)(w[i] & kMask48));
            else acc += chunk_value(w[i] & kMask48, pos & 1);
            pend &= ~(1u << i);
          }
        }
        if (!pend) break;
        if ((it & 31u) == 0u && give_up(a.sync, a.cancel, t0, a.timeout_ticks, it)) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  sacc[tid] = acc;
  if (__syncthreads_or(!ok)) return false;
  if (tid < NV) {
    long long c0 = 0, c1 = 0;
    for (int gg = 0; gg < G; ++gg) {
      c0 += sacc[gg * W + 2 * tid];
      c1 += sacc[gg * W + 2 * tid + 1];
    }
    const I128 tot = i128_add(I128{(unsigned long long)c0, 0ll},
                              I128{(unsigned long long)c1 << 48, c1 >> 16});
    sJ[tid] = i128_to_double(tot) * ((tid / (NV / NM)) == 1 ? a.p2e1 : a.p2e0);
  } else if (MAXE && tid == NV) {
    long long f = 0;
    for (int gg = 0; gg < G; ++gg) f = max(f, sacc[gg * W + 2 * NV]);
    *sE = as_double((unsigned long long)f << 16);
  }
  __syncthreads();
  return true;
}

// Fold the waves' per-lane totals (lane v holds value v) and run the grid reduction.
// MAXE: also the largest of the lanes' error estimates emax (then swm holds one double per
// wave and the grid's largest estimate lands in *sE).  BS: threads per block.
// (always inlined: a call would take the address of the launch arguments and make the
// compiler keep a private copy of them)
template <int NV, bool MAXE, int NM, int BS>
__device__ __forceinline__ bool finish_stage_bs(const StepArgs& a, unsigned epoch, I128 T, I128 (*sw)[NV],
                                long long* sacc, double* sJ, double emax, double* swm, double* sE) {
  constexpr int WPB = BS / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane < NV) sw[wid][lane] = T;
  if constexpr (MAXE) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(emax, off, 64);
      emax = (o > emax) ? o : emax;
    }
    if (lane == 0) swm[wid] = emax;
  }
  __syncthreads();
  I128 blk = i128_zero();
  long long own = 0;
  unsigned long long efield = 0;
  if (threadIdx.x < NV)
    for (int w = 0; w < WPB; ++w) blk = i128_add(blk, sw[w][threadIdx.x]);
  if (blockIdx.x == 0 && threadIdx.x < 2 * NV) {
    I128 c = i128_zero();
    for (int w = 0; w < WPB; ++w) c = i128_add(c, sw[w][threadIdx.x >> 1]);
    own = chunk_value(chunk_field(c, threadIdx.x & 1), threadIdx.x & 1);
  }
  if constexpr (MAXE) {
    if (threadIdx.x == NV || (blockIdx.x == 0 && threadIdx.x == 2 * NV)) {
      double m = 0.0;
      for (int w = 0; w < WPB; ++w) m = (swm[w] > m) ? swm[w] : m;
      efield = as_bits(m) >> 16;
      if (threadIdx.x == 2 * NV) own = (long long)efield;
    }
  }
  return grid_reduce<NV, MAXE, NM, BS>(a, epoch, blk, own, efield, sJ, sacc, sE);
}


// Radii and length of one step: stage radii r0, rm = r0 + h/2 and r1.  On the fixed grid
// r1 = r_start + (n + 1) h (not r0 + h), as in the serial definition.
struct StepGeo {
  double r0, rm, r1, h;
};
__device__ __forceinline__ StepGeo geo_fixed(const StepArgs& a, long long n) {
  StepGeo g;
  g.r0 = a.rs + (double)n * a.h;
  g.rm = g.r0 + 0.5 * a.h;
  g.r1 = a.rs + (double)(n + 1) * a.h;
  g.h = a.h;
  return g;
}

// ------------------------------------------------------------- row helpers
// Fixed-point scales of one model: 2^e1, 2^e0, 2^-e1, 2^-e0.
struct Scales {
  double s1, s0, p2e1, p2e0;
};
// Start value of a lane's 64-bit sums over the segment k0, k0 + 64, ... < kend: minus
// kFixMagic once per contribution (modulo 2^64), so that adding the contributions' bit
// patterns leaves the sum of their integers.
__device__ __forceinline__ unsigned long long fix_base(int k0, int kend) {
  const unsigned long long n = (kend > k0) ? (unsigned long long)((kend - k0 + 63) >> 6) : 0ull;
  return 0ull - n * kFixMagic;
}
// End of a row segment: the lanes' 64-bit sums -> exact per-component wave sums, added to
// `mine` of lanes v < 2 NC (component v % NC).  Through this wave's LDS scratch fl
// ((NC + 2) x 64 words): every lane stores its NC sums; lane (g, c) of G = 64/NC groups adds
// component c of L = ceil(64/G) lanes as a 128-bit integer; lanes v < 2 NC add the G group
// sums of component v % NC.  Integer sums, so the order does not matter.
template <int NC, int NM = 2>
__device__ __forceinline__ void fold_segment(const long long* acc, int lane, long long* fl, I128& mine) {
  // Every lane sum is below 2^56 in magnitude (at most 32 contributions below 2^51, or a
  // mixed-precision lane sum converted below 2^56), so one component's 64 lane sums add up
  // below 2^62: plain 64-bit integer sums, widened to 128 bits once per segment.
  constexpr int G = 64 / NC, L = (64 + G - 1) / G;
#pragma unroll
  for (int i = 0; i < NC; ++i) fl[i * 64 + lane] = acc[i];
  __asm__ volatile("" ::: "memory");   // the wave's LDS operations complete in program order
  long long* gs = fl + NC * 64;
  const int c = lane % NC, g = lane / NC;
  if (g < G) {
    long long part = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int src = g * L + i;
      if (src < 64) part += fl[c * 64 + src];
    }
    gs[g * NC + c] = part;
  }
  __asm__ volatile("" ::: "memory");
  if (lane < NM * NC) {
    const int cc = lane % NC;
    long long t = 0;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) t += gs[gg * NC + cc];
    mine = i128_add(mine, i128_from(t));
  }
  __asm__ volatile("" ::: "memory");
}
// End of a row: lanes v < NC add the J0 angle term (energy sum / cos), lanes
// NC <= v < 2 NC the J1 energy sum, to their running totals; with NM = 4 (extended model)
// lanes 2 NC <= v < 3 NC add the J_sc term (energy sum sin(theta) cos(phi) / cos: asc =
// (sin(theta) / cos) cos(phi)) and 3 NC <= v < 4 NC the J_ss term (ass, sin(phi)).
template <int NC, int NM = 2>
__device__ __forceinline__ void close_row(const Scales& sc, int lane, const I128& mine,
                                          double icmom, I128& T, int& err, double asc = 0.0,
                                          double ass = 0.0) {
  if (lane < NC) {
    T = i128_add(T, i128_from(to_fix(icmom * (i128_to_double(mine) * sc.p2e1), sc.s0, kTwo62, err)));
  } else if (lane < 2 * NC) {
    T = i128_add(T, mine);
  } else if (NM == 4 && lane < 4 * NC) {
    const double f = (lane < 3 * NC) ? asc : ass;
    T = i128_add(T, i128_from(to_fix(f * (i128_to_double(mine) * sc.p2e1), sc.s0, kTwo62, err)));
  }
}

// Row geometry of a stage: cos(theta) and h / cos(theta) at the three stage radii, 1/cos at
// the radius of the stage's moments, and (extended model) sin(theta) at the three radii.
// The wavefront's first row keeps it in LDS (gc, 11 doubles: c0 cm c1 hc0 hcm hc1, 1/cm,
// 1/c1, sin(theta)) from stage 1 of a step for stages 2-4, which use the same radii.
template <int KIND, bool EXT>
__device__ __forceinline__ void stage_geo(double u, double h, const Radial& g0, const Radial& gm,
                                          const Radial& g1, double* gc, RowGeo& rg, double& icmom,
                                          double& sn0, double& snm, double& sn1) {
  if (KIND >= 2 && gc) {
    rg.c0 = gc[0]; rg.cm = gc[1]; rg.c1 = gc[2];
    rg.hc0 = gc[3]; rg.hcm = gc[4]; rg.hc1 = gc[5];
    icmom = (KIND == 2) ? gc[6] : gc[7];
    sn0 = gc[8]; snm = gc[9]; sn1 = gc[10];
    return;
  }
  rg = row_geo(u, h, g0, gm, g1);
  icmom = 1.0 / ((KIND == 0) ? rg.c0 : ((KIND <= 2) ? rg.cm : rg.c1));
  // sin(theta) at the three stage radii (sin(theta) r = sin(theta_R) R)
  sn0 = EXT ? sqrt(u * g0.q2) : 0.0;
  snm = EXT ? sqrt(u * gm.q2) : 0.0;
  sn1 = EXT ? sqrt(u * g1.q2) : 0.0;
  if (KIND == 1 && gc) {
    gc[0] = rg.c0; gc[1] = rg.cm; gc[2] = rg.c1;
    gc[3] = rg.hc0; gc[4] = rg.hcm; gc[5] = rg.hc1;
    gc[6] = icmom;
    gc[7] = 1.0 / rg.c1;
    gc[8] = sn0; gc[9] = snm; gc[10] = sn1;
  }
}

// ----------------------------------------------------------------- two flavours
// Every two-flavour stage keeps its stage-wide and per-row constants in a per-wavefront LDS
// block, written by lane 0 and re-read where they are used, so that the beam loop holds
// only per-beam values in registers (which lets four wavefronts share a SIMD):
constexpr int kC2Rad = 0;    // q2, lam, mu at the stage radii r0, rm, r1 (9)
constexpr int kC2Sc = 9;     // fixed-point scales s1, s0, p2e1, p2e0 (4)
constexpr int kC2Row = 13;   // generator i = 1..4: h/cos, lam, nu-nu term (3): 5 each (20);
                             // then 1/cos at the moments' radius and the azimuthal factors (3)
constexpr int kC2Geo = 36;   // the wavefront's first row's stage geometry (11, stage_geo)
constexpr int kC2Size = 48;
// Stage-wide constants: the radial profiles at the three stage radii and the scales.
__device__ __forceinline__ void put_stage2(double* cb, int lane, const Radial& g0, const Radial& gm,
                                           const Radial& g1, const Scales& sc) {
  if (lane == 0) {
    cb[kC2Rad + 0] = g0.q2; cb[kC2Rad + 1] = g0.lam; cb[kC2Rad + 2] = g0.mu;
    cb[kC2Rad + 3] = gm.q2; cb[kC2Rad + 4] = gm.lam; cb[kC2Rad + 5] = gm.mu;
    cb[kC2Rad + 6] = g1.q2; cb[kC2Rad + 7] = g1.lam; cb[kC2Rad + 8] = g1.mu;
    cb[kC2Sc + 0] = sc.s1; cb[kC2Sc + 1] = sc.s0; cb[kC2Sc + 2] = sc.p2e1; cb[kC2Sc + 3] = sc.p2e0;
  }
  __asm__ volatile("" ::: "memory");   // the wave's LDS operations complete in program order
}
// Stage generator i of beam (bx, bz) from its row constants c = [h/cos, lam, nu-nu term]
// (the arithmetic of gen2).
__device__ __forceinline__ void gen2c(int an, double bx, double bz, const double* c, double f[3]) {
  const double nn[3] = {c[2], c[3], c[4]};
  gen2(an, bx, bz, c[1], nn, c[0], f);
}

// The constants of one row for a stage (the arithmetic every beam of the row shares):
// rc[5 (i - 1) ...] = h/cos, lam and the nu-nu term (3) of stage generator i, then rc[20] =
// 1/cos at the moments' radius and rc[21..22] the extended model's azimuthal factors.
// gcache: the wavefront's first-row geometry slot (or nullptr).  Values are written to rc
// only where write is true.
template <int KIND, bool EXT>
__device__ __forceinline__ void row_setup2(double u, double h, double* cb, const double* const* J,
                                           double cp, double sp, double* gcache, bool write, double* rc) {
  const Radial g0{cb[kC2Rad + 0], cb[kC2Rad + 1], cb[kC2Rad + 2], 0.0};
  const Radial gm{cb[kC2Rad + 3], cb[kC2Rad + 4], cb[kC2Rad + 5], 0.0};
  const Radial g1{cb[kC2Rad + 6], cb[kC2Rad + 7], cb[kC2Rad + 8], 0.0};
  RowGeo rg;
  double icmom, sn0, snm, sn1;
  stage_geo<KIND, EXT>(u, h, g0, gm, g1, gcache, rg, icmom, sn0, snm, sn1);
  double n[3];
  if (KIND == 1 || KIND == 2 || KIND == 4) {
    nunu_row<3, EXT>(J[0], g0.mu, rg.c0, sn0, cp, sp, n);
    if (write) { rc[0] = rg.hc0; rc[1] = g0.lam; rc[2] = n[0]; rc[3] = n[1]; rc[4] = n[2]; }
  }
  if (KIND == 2 || KIND == 4) {
    nunu_row<3, EXT>(J[1], gm.mu, rg.cm, snm, cp, sp, n);
    if (write) { rc[5] = rg.hcm; rc[6] = gm.lam; rc[7] = n[0]; rc[8] = n[1]; rc[9] = n[2]; }
  }
  if (KIND >= 3) {
    nunu_row<3, EXT>(J[2], gm.mu, rg.cm, snm, cp, sp, n);
    if (write) { rc[10] = rg.hcm; rc[11] = gm.lam; rc[12] = n[0]; rc[13] = n[1]; rc[14] = n[2]; }
  }
  if (KIND == 4) {
    nunu_row<3, EXT>(J[3], g1.mu, rg.c1, sn1, cp, sp, n);
    if (write) { rc[15] = rg.hc1; rc[16] = g1.lam; rc[17] = n[0]; rc[18] = n[1]; rc[19] = n[2]; }
  }
  const double snmom = (KIND == 0) ? sn0 : ((KIND <= 2) ? snm : sn1);
  if (write) { rc[20] = icmom; rc[21] = (snmom * icmom) * cp; rc[22] = (snmom * icmom) * sp; }
}
constexpr int kRowC = 26;    // doubles per row-constant block (25 used)

// Stage stencil for one (species s, emission bin u) row of NE beams starting at beam rb.
// KIND: 0 moments of rho_n at r_n; 1 stage Y2 (moments at r_n + h/2); 2 stage Y3
// (r_n + h/2); 3 stage Y4 (r_{n+1}); 4 final update, store and moments at r_{n+1}.
// J[i]: stage moments J^(i+1) (J0 | J1, 6 doubles).  A lane adds the fixed-point
// contributions of up to 32 of its beams in 64-bit integers (each below 2^51) before they
// are folded into exact 128-bit wave sums; a beam whose state has squared norm 2 or more
// (NaN included) sets err.  cb: the wavefront's constant block (put_stage2 written).
// ADAPT (final update only): the new state goes to Xo instead of X, and emax keeps the
// largest embedded error estimate |Theta - f2|^2 of the lane's beams.
// EXT: extended bulb model, azimuth (cp, sp) = (cos, sin) of the row's azimuthal bin.
// geo: this row is the wavefront's first (its stage geometry is cached across stages).
// PRE: the row's constants were computed beforehand (row_setup2) and sit at rcp.
template <int KIND, bool ADAPT = false, bool EXT = false, bool PRE = false>
__device__ __forceinline__ void row2(const double* X, double* Xo, long long plane, long long rb, int NE,
                                     int s, double u, double h, const double* tab, double* cb,
                                     const double* const* J, int renorm, int lane, long long* fl, I128& T,
                                     int& err, double& emax, double cp = 0.0, double sp = 0.0,
                                     int an = -1, bool geo = false, const double* sct = nullptr,
                                     double* rcp = nullptr) {
  // sct: the block's sin/cos constants (sincos_coefs, in LDS)
  constexpr int NM = EXT ? 4 : 2;
  // the lane's first beam of the row, loaded before the row set-up so that the set-up
  // arithmetic overlaps the load
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  if (lane < NE) {
    q0 = X[rb + lane]; q1 = X[rb + lane + plane]; q2 = X[rb + lane + 2 * plane];
  }
  // species row s, antiparticle flag an (default: s itself, two tracked species)
  if (an < 0) an = s;
  double* rc = PRE ? rcp : cb + kC2Row;
  __asm__ volatile("" ::: "memory");   // stage constants re-read from LDS for every row
  if constexpr (!PRE)
    row_setup2<KIND, EXT>(u, h, cb, J, cp, sp, geo ? cb + kC2Geo : nullptr, lane == 0, rc);
  __asm__ volatile("" ::: "memory");
  const double* G = tab + (size_t)(2 + s) * NE;
  I128 mine = i128_zero();
  for (int k0 = lane; k0 - lane < NE; k0 += 64 * 32) {
    const int kend = min(NE, k0 + 64 * 32);
    const unsigned long long base = fix_base(k0, kend);
    unsigned long long acc[3] = {base, base, base};
    if (k0 != lane && k0 < kend) {   // a later segment's first beam
      q0 = X[rb + k0]; q1 = X[rb + k0 + plane]; q2 = X[rb + k0 + 2 * plane];
    }
    for (int k = k0; k < kend; k += 64) {
      double P0 = q0, P1 = q1, P2 = q2;
      if (k + 64 < kend) {    // prefetch the lane's next beam
        q0 = X[rb + k + 64]; q1 = X[rb + k + 64 + plane]; q2 = X[rb + k + 64 + 2 * plane];
      }
      __asm__ volatile("" ::: "memory");   // the row constants are re-read from LDS per beam
      if (KIND >= 1) {
        const double bx = tab[k], bz = tab[NE + k];
        double f1[3], f2[3], f3[3], f4[3];
        if (KIND != 3) gen2c(an, bx, bz, rc + 0, f1);
        if (KIND == 1) {
          rotate2<true>(0.5 * f1[0], 0.5 * f1[1], 0.5 * f1[2], P0, P1, P2, sct);
        } else if (KIND == 2) {
          gen2c(an, bx, bz, rc + 5, f2);
          const double cr0 = f1[1] * f2[2] - f1[2] * f2[1];
          const double cr1 = f1[2] * f2[0] - f1[0] * f2[2];
          const double cr2 = f1[0] * f2[1] - f1[1] * f2[0];
          rotate2<true>(0.5 * f2[0] - 0.125 * cr0, 0.5 * f2[1] - 0.125 * cr1, 0.5 * f2[2] - 0.125 * cr2,
                  P0, P1, P2, sct);
        } else if (KIND == 3) {
          gen2c(an, bx, bz, rc + 10, f3);
          rotate2<true>(f3[0], f3[1], f3[2], P0, P1, P2, sct);
        } else {
          gen2c(an, bx, bz, rc + 5, f2);
          gen2c(an, bx, bz, rc + 10, f3);
          gen2c(an, bx, bz, rc + 15, f4);
          const double cr0 = f1[1] * f4[2] - f1[2] * f4[1];
          const double cr1 = f1[2] * f4[0] - f1[0] * f4[2];
          const double cr2 = f1[0] * f4[1] - f1[1] * f4[0];
          const double t0 = (((f1[0] + 2.0 * f2[0]) + 2.0 * f3[0]) + f4[0]) * (1.0 / 6.0) - cr0 * (1.0 / 12.0);
          const double t1 = (((f1[1] + 2.0 * f2[1]) + 2.0 * f3[1]) + f4[1]) * (1.0 / 6.0) - cr1 * (1.0 / 12.0);
          const double t2 = (((f1[2] + 2.0 * f2[2]) + 2.0 * f3[2]) + f4[2]) * (1.0 / 6.0) - cr2 * (1.0 / 12.0);
          if (ADAPT) {
            const double d0 = t0 - f2[0], d1 = t1 - f2[1], d2 = t2 - f2[2];
            const double e = (d0 * d0 + d1 * d1) + d2 * d2;
            emax = (e > emax) ? e : emax;
          }
          rotate2<true>(t0, t1, t2, P0, P1, P2, sct);
          if (renorm) {
            const double nrm2 = (P0 * P0 + P1 * P1) + P2 * P2;
            if (!(fabs(nrm2 - 1.0) <= kRenormTol)) err |= 8;
            const double inv = fma(-0.5, nrm2, 1.5);   // one Newton step for 1/sqrt from 1
            P0 = P0 * inv;
            P1 = P1 * inv;
            P2 = P2 * inv;
          }
          Xo[rb + k] = P0;
          Xo[rb + k + plane] = P1;
          Xo[rb + k + 2 * plane] = P2;
        }
      }
      // rho~: rho for neutrinos, -rho^* (Bloch (-x, y, -z)) for antineutrinos
      if (!(fma(P0, P0, fma(P1, P1, P2 * P2)) < 2.0)) err |= 1;
      const double ws = G[k] * cb[kC2Sc + 0];
      const double wa = an ? -ws : ws;
      acc[0] += fix_bits(P0, wa);
      acc[1] += fix_bits(P1, ws);
      acc[2] += fix_bits(P2, wa);
    }
    fold_segment<3, NM>(reinterpret_cast<const long long*>(acc), lane, fl, mine);
  }
  __asm__ volatile("" ::: "memory");
  close_row<3, NM>(Scales{cb[kC2Sc + 0], cb[kC2Sc + 1], cb[kC2Sc + 2], cb[kC2Sc + 3]}, lane, mine, rc[20], T,
                   err, rc[21], rc[22]);
}

// A group of gn rows of one model whose beams are contiguous from beam gb0 (NE energies a
// row), streamed as full 64-lane chunks: lane l of chunk c takes the group's beam
// f = 64 c + l, row i = f / NE, energy k = f - i NE, and reads its row's constants from the
// group table rt (row i's block; [kRowS] = species row, [kRowA] = antiparticle flag).  The
// last chunk of one row and the first of the next share a wavefront instead of leaving
// lanes idle.  A row's exact sum is folded in the chunk where the row ends (its lanes fold,
// the others go on with the next row), so every row adds the same integer sum as in row2
// and the moments keep their bits.  A lane adds at most ceil(NE / 64) + 1 contributions
// to a row, so with NE <= kGroupMaxNE its 64-bit sums stay below 2^56 as fold_segment needs.
constexpr int kRowS = 23, kRowA = 24;
constexpr int kGroupMaxNE = 64 * 31;
// Rows folded together by group2.  The extended model's rows (100 energies) end in most
// chunks, and a fold and close of one row costs about as many issue slots as of four, so its
// wavefront folds four rows at a time (60M beams: 2.79 -> 2.45 ms per step).  The batch
// kernel folds one: its rows are longer (50-400 energies) and at 128 VGPRs the staged
// totals spill (two rows at a time: 2.88 -> 4.63 ms).
constexpr int kFoldRowsExt = 4, kFoldRowsBatch = 1;
// A wavefront's fold scratch for group2 with R rows per fold: 3 R staged components, each
// in a run of fold2_stride(R) words, then the 3 R G partial sums (G = 64 / 3 R per
// component).  With R > 1 a run is 64 + G words and lane g of component c adds words g,
// g + G, ...: the padding puts component c's run G banks after component c - 1's, so these
// reads meet no bank conflicts (the extended model's 12 components would otherwise read
// one bank 12-fold; 60M beams 2.43 -> 2.35 ms per step).  With R = 1 (3 components) the
// plain layout is kept: its index arithmetic costs the batch kernel more in spills than
// the conflicts (2.89 against 3.04 ms).
__host__ __device__ constexpr int fold2_stride(int R) { return (R > 1) ? 64 + 64 / (3 * R) : 64; }
__host__ __device__ constexpr int fold2_words(int R) { return 3 * R * fold2_stride(R) + 64; }

// Fold of up to R rows whose lane sums were staged as they ended: component c of slot q in
// fl[(q * 3 + c) * S + lane], q < nrows, S = fold2_stride(R).  The same integer reduction as
// fold_segment over 3 R components at once: G partial sums per component, each over every
// G-th word (R > 1) or over a run of words (R = 1), then lane v adds the G partial sums of
// its component.  Lane m * 3 R + q * 3 + c then closes moment m, component c of the row in
// slot q (its row constants at rr0 + q * kRowC) exactly as close_row does, into Tq.  One
// set of instructions folds and closes R rows, instead of one per row.
template <int R, int NM>
__device__ __forceinline__ void fold_rows2(int lane, long long* fl, int nrows, const double* rr0,
                                           const Scales& sc, I128& Tq, int& err) {
  constexpr int NCR = 3 * R, G = 64 / NCR, L = (64 + G - 1) / G, S = fold2_stride(R);
  constexpr bool PAD = R > 1;
  long long* gs = fl + NCR * S;
  __asm__ volatile("" ::: "memory");   // the wave's LDS operations complete in program order
  // lane (cc, g): partial sum g of component cc, stored at gs[cc * G + g] (R > 1) or
  // gs[g * NCR + cc] (R = 1)
  if (PAD) {
    const int cc = lane / G, g = lane - cc * G;
    if (cc < NCR) {
      long long part = 0;
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const int src = i * G + g;
        if (src < 64) part += fl[cc * S + src];
      }
      gs[cc * G + g] = part;
    }
  } else {
    const int cc = lane % NCR, g = lane / NCR;
    if (g < G) {
      long long part = 0;
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const int src = g * L + i;
        if (src < 64) part += fl[cc * S + src];
      }
      gs[g * NCR + cc] = part;
    }
  }
  __asm__ volatile("" ::: "memory");
  if (lane < NM * NCR) {
    const int m = lane / NCR, qc = lane - m * NCR, q = qc / 3;
    if (q < nrows) {
      long long t = 0;
#pragma unroll
      for (int gg = 0; gg < G; ++gg) t += gs[PAD ? qc * G + gg : gg * NCR + qc];
      const double* rr = rr0 + q * kRowC;
      if (m == 1) {
        Tq = i128_add(Tq, i128_from(t));
      } else {
        const double f = (m == 0) ? rr[20] : ((m == 2) ? rr[21] : rr[22]);
        Tq = i128_add(Tq, i128_from(to_fix(f * (i128_to_double(i128_from(t)) * sc.p2e1), sc.s0, kTwo62, err)));
      }
    }
  }
  __asm__ volatile("" ::: "memory");
}

template <int KIND, bool EXT, int R>
__device__ __forceinline__ void group2(double* X, long long plane, long long gb0, int NE, int gn,
                                       const double* tab, double* cb, const double* rt, int renorm,
                                       int lane, long long* fl, I128& T, int& err, const double* sct) {
  constexpr int NM = EXT ? 4 : 2;
  constexpr int NCR = 3 * R, S = fold2_stride(R);
  const Scales sc{cb[kC2Sc + 0], cb[kC2Sc + 1], cb[kC2Sc + 2], cb[kC2Sc + 3]};
  const int nbeam = gn * NE;
  const int nchunk = (nbeam + 63) >> 6;
  int i = lane / NE;                 // the lane's row and energy in the current chunk
  int k = lane - i * NE;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  // PF (batches): the energy tables of a batch's models stay in HBM, so the lane's table
  // values (vacuum terms and weight) for its beam in the next chunk are loaded with that
  // beam's state, instead of at their use (256-model batch 2.90 -> 2.53 ms per step).  The
  // extended model reads its tables from LDS.
  constexpr bool PF = !EXT;
  double tx = 0.0, tz = 0.0, tw = 0.0;
  if (lane < nbeam) {
    q0 = X[gb0 + lane]; q1 = X[gb0 + lane + plane]; q2 = X[gb0 + lane + 2 * plane];
    if (PF) {
      tx = tab[k]; tz = tab[NE + k]; tw = tab[(size_t)(2 + (int)rt[i * kRowC + kRowS]) * NE + k];
    }
  }
  unsigned long long acc[3] = {0ull, 0ull, 0ull};
  unsigned long long cnt = 0;        // contributions in acc (each carries kFixMagic)
  int r = 0;                         // the oldest unfinished row (wave-uniform)
  int ns = 0;                        // ended rows staged for the next fold (wave-uniform)
  I128 Tq = i128_zero();             // closed rows, lane m * 3 R + q * 3 + c (fold_rows2)
  for (int c = 0; c < nchunk; ++c) {
    const int f = (c << 6) + lane;
    const bool on = f < nbeam;
    double P0 = q0, P1 = q1, P2 = q2;
    const double bxc = tx, bzc = tz, wsc = tw;
    if (f + 64 < nbeam) {    // prefetch the lane's next beam
      q0 = X[gb0 + f + 64]; q1 = X[gb0 + f + 64 + plane]; q2 = X[gb0 + f + 64 + 2 * plane];
      if (PF) {
        int k2 = k + 64, i2 = i;
        while (k2 >= NE) {
          k2 -= NE;
          ++i2;
        }
        tx = tab[k2]; tz = tab[NE + k2]; tw = tab[(size_t)(2 + (int)rt[i2 * kRowC + kRowS]) * NE + k2];
      }
    }
    __asm__ volatile("" ::: "memory");   // the row constants are re-read from LDS per beam
    unsigned long long x0 = 0ull, x1 = 0ull, x2 = 0ull;
    if (on) {
      const double* rc = rt + i * kRowC;
      const int sr = (int)rc[kRowS], an = (int)rc[kRowA];
      if (KIND >= 1) {
        const double bx = PF ? bxc : tab[k], bz = PF ? bzc : tab[NE + k];
        double f1[3], f2[3], f3[3], f4[3];
        if (KIND != 3) gen2c(an, bx, bz, rc + 0, f1);
        if (KIND == 1) {
          rotate2<true>(0.5 * f1[0], 0.5 * f1[1], 0.5 * f1[2], P0, P1, P2, sct);
        } else if (KIND == 2) {
          gen2c(an, bx, bz, rc + 5, f2);
          const double cr0 = f1[1] * f2[2] - f1[2] * f2[1];
          const double cr1 = f1[2] * f2[0] - f1[0] * f2[2];
          const double cr2 = f1[0] * f2[1] - f1[1] * f2[0];
          rotate2<true>(0.5 * f2[0] - 0.125 * cr0, 0.5 * f2[1] - 0.125 * cr1, 0.5 * f2[2] - 0.125 * cr2,
                        P0, P1, P2, sct);
        } else if (KIND == 3) {
          gen2c(an, bx, bz, rc + 10, f3);
          rotate2<true>(f3[0], f3[1], f3[2], P0, P1, P2, sct);
        } else {
          gen2c(an, bx, bz, rc + 5, f2);
          gen2c(an, bx, bz, rc + 10, f3);
          gen2c(an, bx, bz, rc + 15, f4);
          const double cr0 = f1[1] * f4[2] - f1[2] * f4[1];
          const double cr1 = f1[2] * f4[0] - f1[0] * f4[2];
          const double cr2 = f1[0] * f4[1] - f1[1] * f4[0];
          const double t0 = (((f1[0] + 2.0 * f2[0]) + 2.0 * f3[0]) + f4[0]) * (1.0 / 6.0) - cr0 * (1.0 / 12.0);
          const double t1 = (((f1[1] + 2.0 * f2[1]) + 2.0 * f3[1]) + f4[1]) * (1.0 / 6.0) - cr1 * (1.0 / 12.0);
          const double t2 = (((f1[2] + 2.0 * f2[2]) + 2.0 * f3[2]) + f4[2]) * (1.0 / 6.0) - cr2 * (1.0 / 12.0);
          rotate2<true>(t0, t1, t2, P0, P1, P2, sct);
          if (renorm) {
            const double nrm2 = (P0 * P0 + P1 * P1) + P2 * P2;
            if (!(fabs(nrm2 - 1.0) <= kRenormTol)) err |= 8;
            const double inv = fma(-0.5, nrm2, 1.5);   // one Newton step for 1/sqrt from 1
            P0 = P0 * inv;
            P1 = P1 * inv;
            P2 = P2 * inv;
          }
          X[gb0 + f] = P0;
          X[gb0 + f + plane] = P1;
          X[gb0 + f + 2 * plane] = P2;
        }
      }
      // rho~: rho for neutrinos, -rho^* (Bloch (-x, y, -z)) for antineutrinos
      if (!(fma(P0, P0, fma(P1, P1, P2 * P2)) < 2.0)) err |= 1;
      const double ws = (PF ? wsc : tab[(size_t)(2 + sr) * NE + k]) * cb[kC2Sc + 0];
      const double wa = an ? -ws : ws;
      x0 = fix_bits(P0, wa);
      x1 = fix_bits(P1, ws);
      x2 = fix_bits(P2, wa);
    }
    // stage every row that ends in this chunk (its lanes add their contribution first);
    // fold R staged rows at a time
    const int fend = min(nbeam, (c + 1) << 6);
    while (r < gn && (r + 1) * NE <= fend) {
      if (on && i == r) {
        acc[0] += x0; acc[1] += x1; acc[2] += x2;
        ++cnt;
      }
      const unsigned long long bias = cnt * kFixMagic;
      long long* slot = fl + ns * 3 * S + lane;
      slot[0] = (long long)(acc[0] - bias);
      slot[S] = (long long)(acc[1] - bias);
      slot[2 * S] = (long long)(acc[2] - bias);
      acc[0] = acc[1] = acc[2] = 0ull;
      cnt = 0;
      ++r;
      if (++ns == R) {
        fold_rows2<R, NM>(lane, fl, R, rt + (r - R) * kRowC, sc, Tq, err);
        ns = 0;
      }
    }
    if (on && i == r) {      // the row that goes on into the next chunk
      acc[0] += x0; acc[1] += x1; acc[2] += x2;
      ++cnt;
    }
    k += 64;                 // the lane's beam in the next chunk
    while (k >= NE) {
      k -= NE;
      ++i;
    }
  }
  if (ns) fold_rows2<R, NM>(lane, fl, ns, rt + (r - ns) * kRowC, sc, Tq, err);
  // the closed rows' totals (lane m * 3 R + q * 3 + c) into T (lane m * 3 + c): integer sums
  __asm__ volatile("" ::: "memory");
  if (lane < NM * NCR) {
    fl[2 * lane] = (long long)Tq.lo;
    fl[2 * lane + 1] = Tq.hi;
  }
  __asm__ volatile("" ::: "memory");
  if (lane < NM * 3) {
    const int m = lane / 3, c = lane - 3 * m;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int src = m * NCR + q * 3 + c;
      T = i128_add(T, I128{(unsigned long long)fl[2 * src], fl[2 * src + 1]});
    }
  }
  __asm__ volatile("" ::: "memory");
}

// rt (extended model): the wavefront's row-constant table of kGroup2 blocks of kRowC.
constexpr int kGroup2 = 16;
template <int KIND, bool ADAPT = false, bool EXT = false>
__device__ __forceinline__ void stage2(const StepArgs& a, const StepGeo& G, const double* X, double* Xo,
                                       const double (*sJ)[EXT ? 12 : 6], const double* tab, long long gw,
                                       long long nw, int lane, long long* fl, I128& T, int& err,
                                       double& emax, double* cb, const double* sct, bool geo = false,
                                       double* rt = nullptr) {
  put_stage2(cb, lane, radial_at(a, G.r0), radial_at(a, G.rm), radial_at(a, G.r1),
             Scales{a.s1, a.s0, a.p2e1, a.p2e0});
  const double* J[4] = {sJ[0], sJ[1], sJ[2], sJ[3]};
  if constexpr (EXT) {
    // rows (s, j, p): species, emission bin, azimuthal bin.  Each wavefront takes a
    // contiguous range of rows, in groups of up to kGroup2: lane l computes the constants of
    // the group's row l (row_setup2: geometry, nu-nu terms with the row's azimuth) into the
    // table rt, then the rows run one after the other.
    // (the launch arguments are read into locals first: the LDS-order barriers below would
    // otherwise make the compiler re-read them from a private copy of the argument block)
    const int NE = a.NE, NU = a.NU, NP = a.NP, NS = a.NS, renorm = a.renorm;
    const long long plane = a.plane;
    const double h = G.h;
    const double* phi = a.tab + (size_t)(2 + NS) * NE;
    const long long nrow = (long long)NS * NU * NP;
    const long long per = (nrow + nw - 1) / nw;
    const long long rbeg = gw * per, rend = min(nrow, rbeg + per);
    for (long long row = rbeg; row < rend;) {
      const int gn = (int)min(rend - row, (long long)kGroup2);
      __asm__ volatile("" ::: "memory");   // the previous group's rows have read their blocks
      if (lane < gn) {
        const long long r = row + lane;
        const long long sj = r / NP;
        const int p = (int)(r - sj * NP);
        const int s = (int)(sj / NU);
        const int j = (int)(sj - (long long)s * NU);
        row_setup2<KIND, true>(u_of(j, NU), h, cb, J, phi[p], phi[NP + p], nullptr, true, rt + lane * kRowC);
        rt[lane * kRowC + kRowS] = (double)s;
        rt[lane * kRowC + kRowA] = (double)(s >= (NS >> 1));
      }
      __asm__ volatile("" ::: "memory");
      if (!ADAPT && NE <= kGroupMaxNE) {
        group2<KIND, true, kFoldRowsExt>(Xo, plane, row * NE, NE, gn, tab, cb, rt, renorm, lane, fl, T, err, sct);
        row += gn;
      } else {
        for (int i = 0; i < gn; ++i, ++row) {
          const long long sj = row / NP;
          const int s = (int)(sj / NU);
          row2<KIND, ADAPT, true, true>(X, Xo, plane, row * NE, NE, s, 0.0, h, tab, cb, J, renorm, lane, fl, T,
                                        err, emax, 0.0, 0.0, s >= (NS >> 1), false, sct, rt + i * kRowC);
        }
      }
    }
  } else {
    const long long nrow = (long long)a.NS * a.NU;
    for (long long row = gw; row < nrow; row += nw) {
      const int s = (int)(row / a.NU);
      const int j = (int)(row - (long long)s * a.NU);
      row2<KIND, ADAPT>(X, Xo, a.plane, row * a.NE, a.NE, s, u_of(j, a.NU), G.h, tab, cb, J, a.renorm,
                        lane, fl, T, err, emax, 0.0, 0.0, s >= (a.NS >> 1), geo && row == gw, sct);
    }
  }
}

// --------------------------------------------------------------- three flavours
// Stage generators by linearity.  Stage i's generator of a beam of energy bin k is
// K_i = a_i (V_k + M_i): a_i = h / cos(theta) at the stage radius, V_k = e_k V0 the vacuum
// Hamiltonian of the bin (e_k = 1 / E_k), M_i the matter and nu-nu part, the same for
// every energy of a (species, angle) row.  Every generator the step exponentiates is
// affine in V_k; with i[K_1, K_i] = a_1 a_i (e_k i[V0, D] + i[M_1, D]), D = M_i - M_1, each
// is G = alpha V_k + e_k P + Q with alpha, P, Q fixed per row:
//   K1/2               alpha = a1/2, P = 0, Q = (a1/2) M1
//   K3                 alpha = am,   P = 0, Q = am M3
//   K2/2 + i[K1,K2]/8  alpha = am/2, P = c i[V0, D], Q = (am/2) M2 + c i[M1, D], c = a1 am/8
//   Theta              alpha = (a1 + 2 am + 2 am + a4)/6, P = c i[V0, D],
//                      Q = S/6 + c i[M1, D], c = a1 a4/12, S = a1 M1 + 2 am M2 + 2 am M3 + a4 M4
// and the error estimate Theta - K2 = (alpha - am) V_k + e_k P + (Q - am M2).  Per beam that
// is 6 (no P) or 15 fma.  Hermitian matrices as 9 reals: d0 d1 d2, re/im of (0,1), (0,2),
// (1,2).
// alpha V_k + Q
__device__ __forceinline__ Herm3 lin3q(double alpha, const double* Q, const double* v) {
  return Herm3{fma(alpha, v[0], Q[0]), fma(alpha, v[1], Q[1]), fma(alpha, v[2], Q[2]),
               mk(fma(alpha, v[3], Q[3]), Q[4]), mk(fma(alpha, v[4], Q[5]), Q[6]),
               mk(fma(alpha, v[5], Q[7]), Q[8])};
}
// alpha V_k + e_k P + Q
__device__ __forceinline__ Herm3 lin3p(double alpha, const double* P, const double* Q, const double* v,
                                       double ek) {
  return Herm3{fma(alpha, v[0], fma(ek, P[0], Q[0])), fma(alpha, v[1], fma(ek, P[1], Q[1])),
               fma(alpha, v[2], fma(ek, P[2], Q[2])),
               mk(fma(alpha, v[3], fma(ek, P[3], Q[3])), fma(ek, P[4], Q[4])),
               mk(fma(alpha, v[4], fma(ek, P[5], Q[5])), fma(ek, P[6], Q[6])),
               mk(fma(alpha, v[5], fma(ek, P[7], Q[7])), fma(ek, P[8], Q[8]))};
}

// Row constants of stage KIND's generator (KIND >= 1): Q to snn[0..8], P to snn[9..17]
// and, with ADAPT (KIND 4), the error estimate's Q to snn[18..26]; returns alpha (and the
// error estimate's alpha in alphaE).  J0..J3: the stage moments.  Lane i < 9 computes
// component i of every 9-real matrix (the same operations as a matrix-at-a-time
// evaluation, component by component); the commutators read their operands as full
// complex 3x3 matrices from the wavefront's scratch fl (free before the beam loop), where
// each lane writes its component and its mirror.
// Component i of the 9-real form: 0..2 the diagonal, 3 + 2t / 4 + 2t re / im of entry t of
// (0,1), (0,2), (1,2).  nn component of M's component i (the matter part sits on i = 0):
__device__ __forceinline__ int nn_index(int i) { return (i <= 1) ? i : i - 1; }
// nu-nu component j of a row (as nunu_row)
template <int NC, bool EXT>
__device__ __forceinline__ double nunu_comp(const double* J, double mu, double c, double sn, double cp,
                                            double sp, int j) {
  if constexpr (EXT) return mu * ((J[j] - c * J[NC + j]) - sn * (cp * J[2 * NC + j] + sp * J[3 * NC + j]));
  else return mu * (J[j] - c * J[NC + j]);
}
// component i of M = lam E_ee + nn (neutrinos) or -(lam E_ee + nn^*) (antineutrinos)
__device__ __forceinline__ double matter_comp(int an, double lam, double nnv, int i) {
  const double sg = an ? -1.0 : 1.0;
  if (i == 0) return sg * (lam + nnv);
  if (i == 2) return 0.0;
  return (i >= 4 && (i & 1) == 0) ? nnv : sg * nnv;
}
// Write component i of a 9-real Hermitian matrix (value v) into the full complex 3x3
// matrix F (row-major, re/im pairs), with its conjugate mirror.
__device__ __forceinline__ void put_full(double* F, int i, double v) {
  if (i < 3) {
    F[(i * 3 + i) * 2] = v;
    F[(i * 3 + i) * 2 + 1] = 0.0;
  } else {
    const int t = (i - 3) >> 1, a = (t == 2) ? 1 : 0, b = (t == 0) ? 1 : 2;
    if ((i & 1) == 1) {   // real part
      F[(a * 3 + b) * 2] = v;
      F[(b * 3 + a) * 2] = v;
    } else {              // imaginary part
      F[(a * 3 + b) * 2 + 1] = v;
      F[(b * 3 + a) * 2 + 1] = -v;
    }
  }
}
// Component i of i[A, B] from the full matrices (X = A B; C_aa = -2 Im X_aa, C_ab =
// (-(Im X_ab + Im X_ba), Re X_ab - Re X_ba)), as icomm.
__device__ __forceinline__ double icomm_comp(const double* A, const double* B, int i) {
  int a, b;
  if (i < 3) {
    a = i;
    b = i;
  } else {
    const int t = (i - 3) >> 1;
    a = (t == 2) ? 1 : 0;
    b = (t == 0) ? 1 : 2;
  }
  auto at = [](const double* F, int r, int c) { return mk(F[(r * 3 + c) * 2], F[(r * 3 + c) * 2 + 1]); };
  const cplx xab = dot3_mul(at(A, a, 0), at(B, 0, b), at(A, a, 1), at(B, 1, b), at(A, a, 2), at(B, 2, b));
  if (i < 3) return -2.0 * xab.im;
  const cplx xba = dot3_mul(at(A, b, 0), at(B, 0, a), at(A, b, 1), at(B, 1, a), at(A, b, 2), at(B, 2, a));
  if ((i & 1) == 1) return -(xab.im + xba.im);
  return xab.re - xba.re;
}
template <int KIND, bool ADAPT, bool EXT>
__device__ __forceinline__ double row_lin3(const StepArgs& a, int an, const RowGeo& rg, const Radial& g0,
                                           const Radial& gm, const Radial& g1, const double* J0,
                                           const double* J1, const double* J2, const double* J3,
                                           double sn0, double snm, double sn1, double cp, double sp,
                                           double* snn, double& alphaE, int lane, double* scr) {
  constexpr int NC = 8;
  const int i = (lane < 9) ? lane : 8;   // lanes 9..63 repeat component 8 and write nothing
  const int jn = nn_index(i);
  double M1 = 0.0, M2 = 0.0, M3 = 0.0, M4 = 0.0;
  if (KIND != 3) M1 = matter_comp(an, g0.lam, nunu_comp<NC, EXT>(J0, g0.mu, rg.c0, sn0, cp, sp, jn), i);
  if (KIND == 2 || KIND == 4) M2 = matter_comp(an, gm.lam, nunu_comp<NC, EXT>(J1, gm.mu, rg.cm, snm, cp, sp, jn), i);
  if (KIND >= 3) M3 = matter_comp(an, gm.lam, nunu_comp<NC, EXT>(J2, gm.mu, rg.cm, snm, cp, sp, jn), i);
  if (KIND == 4) M4 = matter_comp(an, g1.lam, nunu_comp<NC, EXT>(J3, g1.mu, rg.c1, sn1, cp, sp, jn), i);
  double alpha;
  if (KIND == 1 || KIND == 3) {
    alpha = (KIND == 1) ? 0.5 * rg.hc0 : rg.hcm;
    if (lane < 9) snn[i] = alpha * ((KIND == 1) ? M1 : M3);
  } else {
    const double D = ((KIND == 2) ? M2 : M4) - M1;
    // full matrices: V0 at scr[0..17], M1 at scr[18..35], D at scr[36..53]
    double* FV = scr;
    double* FM = scr + 18;
    double* FD = scr + 36;
    if (lane < 9) {
      const double v0 = (i < 3) ? a.v0[i] : (((i & 1) == 1) ? a.v0[3 + ((i - 3) >> 1)] : 0.0);
      put_full(FV, i, v0);
      put_full(FM, i, M1);
      put_full(FD, i, D);
    }
    __asm__ volatile("" ::: "memory");   // the wave's LDS operations complete in program order
    const double R1 = icomm_comp(FV, FD, i), R2 = icomm_comp(FM, FD, i);
    __asm__ volatile("" ::: "memory");
    if (KIND == 2) {
      const double c = (rg.hc0 * rg.hcm) * 0.125;
      alpha = 0.5 * rg.hcm;
      if (lane < 9) {
        snn[9 + i] = c * R1;
        snn[i] = fma(alpha, M2, c * R2);
      }
    } else {
      const double c = (rg.hc0 * rg.hc1) * (1.0 / 12.0), a2 = 2.0 * rg.hcm;
      alpha = (((rg.hc0 + a2) + a2) + rg.hc1) * (1.0 / 6.0);
      alphaE = alpha - rg.hcm;
      const double S = fma(rg.hc1, M4, fma(a2, M3, fma(a2, M2, rg.hc0 * M1)));
      const double Qi = fma(S, 1.0 / 6.0, c * R2);
      if (lane < 9) {
        snn[9 + i] = c * R1;
        snn[i] = Qi;
        if (ADAPT) snn[18 + i] = fma(-rg.hcm, M2, Qi);
      }
    }
  }
  __asm__ volatile("" ::: "memory");
  return alpha;
}

// The row constants Q, P (and the error estimate's Q) live in LDS (one 32-double block per
// wave) and are re-read per beam, so the compiler does not keep all of them in registers.
// One (species, emission bin) row of the three-flavour stage, FP64 arithmetic.
// ADAPT (final update only): the new state goes to Xo instead of X, and emax keeps the
// largest embedded error estimate |Theta - K2|^2 (traceless part, Frobenius norm).
// EXT: extended bulb model; rows are (s, j, p) with the azimuth table of the tables.
//
// PK (packed row tails; three flavours, FP64 fixed steps, stages 1-4, one row per
// wavefront, 512-thread blocks, N_E = 64 m + t with 1 <= t <= 32 and N_E <= 2048): a row
// takes m full passes and one pass with t busy lanes.  Wavefronts w and w + 4 of a block
// share a SIMD (the placement measured on this device), so wavefront w < 4 (the owner) also
// runs its partner's tail: after its m passes it runs one pass with lanes 0-31 on its own
// beams 64 m + l and lanes 32-63 on the partner's beams 64 m + l - 32 (with the partner's
// row constants), and the SIMD issues 2 m + 1 passes instead of 2 m + 2.  The owner adds its
// tail's contributions to its own lane sums and hands the partner's over through the
// partner's fold scratch flp as exact integers, so every row adds the same integer sum and
// the moments keep their bits.  Block barriers: after the row constants (the owner reads
// its partner's, snp) and before the partner's fold (the handed-over sums).
template <typename ST, int KIND, bool ADAPT = false, bool EXT = false, bool PK = false>
__device__ __forceinline__ void row3(const StepArgs& a, const ST* X, ST* Xo, long long row, double h,
                                     const Radial& g0, const Radial& gm, const Radial& g1,
                                     const double (*sJ)[EXT ? 32 : 16], const double* tab, double* snn,
                                     int lane, long long* fl, I128& T, int& err, double& emax,
                                     const ST* pre = nullptr, double* gc = nullptr, const double* snp = nullptr,
                                     long long* flp = nullptr, bool owner = false) {
  static_assert(!PK || (!ADAPT && !EXT && sizeof(ST) == 8 && KIND >= 1), "packed tails: FP64 fixed steps");
  constexpr int NM = EXT ? 4 : 2;
  const long long plane = a.plane;
  const int NE = a.NE;
  int s, j;
  double cp = 0.0, sp = 0.0;
  if constexpr (EXT) {
    const long long sj = row / a.NP;
    const int p = (int)(row - sj * a.NP);
    s = (int)(sj / a.NU);
    j = (int)(sj - (long long)s * a.NU);
    const double* phi = a.tab + (size_t)(kVacRows3 + a.NS) * a.NE;
    cp = phi[p];
    sp = phi[a.NP + p];
  } else {
    s = (int)(row / a.NU);
    j = (int)(row - (long long)s * a.NU);
  }
  const int an = (s >= (a.NS >> 1)) ? 1 : 0;   // antiparticle row
  const double u = u_of(j, a.NU);
  RowGeo rg;
  double icmom, sn0, snm, sn1;
  stage_geo<KIND, EXT>(u, h, g0, gm, g1, gc, rg, icmom, sn0, snm, sn1);
  double alpha = 0.0, alphaE = 0.0;
  if constexpr (KIND >= 1)
    alpha = row_lin3<KIND, ADAPT, EXT>(a, an, rg, g0, gm, g1, sJ[0], sJ[1], sJ[2], sJ[3], sn0, snm, sn1,
                                       cp, sp, snn, alphaE, lane, reinterpret_cast<double*>(fl));
  if constexpr (PK) {
    if (lane == 0) {
      snn[28] = alpha;
      snn[29] = (double)s;
    }
    __syncthreads();   // every row's constants are in place (the owner reads its partner's)
  }
  const double* G = tab + (size_t)(kVacRows3 + s) * NE;
  const long long rb = row * NE;
  // PK: the full passes end at kmain; the owner's packed pass takes lane l to beam
  // kmain + (l & 31) of its own row (l < 32) or its partner's (row + 4)
  const int kmain = NE & ~63;
  const bool ton = PK && owner && (lane & 31) < NE - kmain;
  const long long rbt = (lane >> 5) ? rb + 4LL * NE : rb;
  I128 mine = i128_zero();
  for (int k0 = lane; k0 - lane < NE; k0 += 64 * 32) {
    const int kend = PK ? kmain : min(NE, k0 + 64 * 32);
    const unsigned long long base = fix_base(k0, kend);
    unsigned long long acc[8] = {base, base, base, base, base, base, base, base};
    ST q[6];
    if (k0 < kend) {
      if (pre && k0 == lane) {   // the lane's first beam, loaded before the last barrier
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = pre[c];
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = X[rb + k0 + c * plane];
      }
    }
    for (int k = k0; k < kend; k += 64) {
      cplx ps[3] = {mk((double)q[0], (double)q[1]), mk((double)q[2], (double)q[3]),
                    mk((double)q[4], (double)q[5])};
      if (k + 64 < kend) {    // prefetch the lane's next beam
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = X[rb + k + 64 + c * plane];
      } else if (PK && ton) {   // the lane's beam of the packed pass
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = X[rbt + kmain + (lane & 31) + c * plane];
      }
      __asm__ volatile("" ::: "memory");   // re-read the row's nn terms from LDS per beam
      if (KIND >= 1) {
        double v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = tab[c * NE + k];
        if (KIND == 1 || KIND == 3) {
          exp3_apply(lin3q(alpha, snn, v), ps);
        } else if (KIND == 2) {
          exp3_apply(lin3p(alpha, snn + 9, snn, v, tab[6 * NE + k]), ps);
        } else {
          const double ek = tab[6 * NE + k];
          const Herm3 Th = lin3p(alpha, snn + 9, snn, v, ek);
          if (ADAPT) {
            // |Theta - K2|^2: traceless part, Frobenius norm
            const Herm3 Ed = lin3p(alphaE, snn + 9, snn + 18, v, ek);
            const double tr = ((Ed.d0 + Ed.d1) + Ed.d2) * (1.0 / 3.0);
            const double a0 = Ed.d0 - tr, a1 = Ed.d1 - tr, a2 = Ed.d2 - tr;
            const double o0 = Ed.o01.re * Ed.o01.re + Ed.o01.im * Ed.o01.im;
            const double o1 = Ed.o02.re * Ed.o02.re + Ed.o02.im * Ed.o02.im;
            const double o2 = Ed.o12.re * Ed.o12.re + Ed.o12.im * Ed.o12.im;
            const double e = ((a0 * a0 + a1 * a1) + a2 * a2) + 2.0 * ((o0 + o1) + o2);
            emax = (e > emax) ? e : emax;
          }
          exp3_apply(Th, ps);
          if (a.renorm) {
            const double nrm2 = (norm2(ps[0]) + norm2(ps[1])) + norm2(ps[2]);
            if (!(fabs(nrm2 - 1.0) <= (sizeof(ST) == 8 ? kRenormTol : kRenormTol32))) err |= 8;
            const double inv = fma(-0.5, nrm2, 1.5);   // one Newton step for 1/sqrt from 1
#pragma unroll
            for (int c = 0; c < 3; ++c) ps[c] = mk(ps[c].re * inv, ps[c].im * inv);
          }
          // store, and take the next step's moments from exactly what was stored
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const ST re = (ST)ps[c].re, im = (ST)ps[c].im;
            Xo[rb + k + (2 * c) * plane] = re;
            Xo[rb + k + (2 * c + 1) * plane] = im;
            ps[c] = mk((double)re, (double)im);
          }
        }
      }
      // rho~ components: rho_ee-rho_tt, rho_mm-rho_tt, Re/Im rho_em, rho_et, rho_mt;
      // antineutrinos: -rho^* (real parts and diagonal negated)
      const double n0 = norm2(ps[0]), nm = norm2(ps[1]), nt = norm2(ps[2]);
      const cplx em = cmul_conjb(ps[0], ps[1]), et = cmul_conjb(ps[0], ps[2]), mt = cmul_conjb(ps[1], ps[2]);
      const double v8[8] = {n0 - nt, nm - nt, em.re, em.im, et.re, et.im, mt.re, mt.im};
      if (!((n0 + nm) + nt < 2.0)) err |= 1;
      const double ws = G[k] * a.s1;
      const double wa = an ? -ws : ws;    // the negated components of -rho^*
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[i] += fix_bits(v8[i], (i < 3 || i == 4 || i == 6) ? wa : ws);
    }
    if constexpr (PK) {
      if (owner) {
        // the packed pass: the same arithmetic as a full pass, with each lane's row constants
        __asm__ volatile("" ::: "memory");
        unsigned long long x[8] = {kFixMagic, kFixMagic, kFixMagic, kFixMagic,
                                   kFixMagic, kFixMagic, kFixMagic, kFixMagic};
        if (ton) {
          const int hf = lane >> 5, k = kmain + (lane & 31);
          const double* sl = hf ? snp : snn;
          const double al = hf ? snp[28] : alpha;
          const int sh = hf ? (int)snp[29] : s;
          const int anl = (sh >= (a.NS >> 1)) ? 1 : 0;
          cplx ps[3] = {mk((double)q[0], (double)q[1]), mk((double)q[2], (double)q[3]),
                        mk((double)q[4], (double)q[5])};
          double v[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) v[c] = tab[c * NE + k];
          if (KIND == 1 || KIND == 3) {
            exp3_apply(lin3q(al, sl, v), ps);
          } else if (KIND == 2) {
            exp3_apply(lin3p(al, sl + 9, sl, v, tab[6 * NE + k]), ps);
          } else {
            const double ek = tab[6 * NE + k];
            exp3_apply(lin3p(al, sl + 9, sl, v, ek), ps);
            if (a.renorm) {
              const double nrm2 = (norm2(ps[0]) + norm2(ps[1])) + norm2(ps[2]);
              if (!(fabs(nrm2 - 1.0) <= kRenormTol)) err |= 8;
              const double inv = fma(-0.5, nrm2, 1.5);   // one Newton step for 1/sqrt from 1
#pragma unroll
              for (int c = 0; c < 3; ++c) ps[c] = mk(ps[c].re * inv, ps[c].im * inv);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              Xo[rbt + k + (2 * c) * plane] = (ST)ps[c].re;
              Xo[rbt + k + (2 * c + 1) * plane] = (ST)ps[c].im;
            }
          }
          const double n0 = norm2(ps[0]), nm = norm2(ps[1]), nt = norm2(ps[2]);
          const cplx em = cmul_conjb(ps[0], ps[1]), et = cmul_conjb(ps[0], ps[2]), mt = cmul_conjb(ps[1], ps[2]);
          const double v8[8] = {n0 - nt, nm - nt, em.re, em.im, et.re, et.im, mt.re, mt.im};
          if (!((n0 + nm) + nt < 2.0)) err |= 1;
          const double ws = tab[(size_t)(kVacRows3 + sh) * NE + k] * a.s1;
          const double wa = anl ? -ws : ws;
#pragma unroll
          for (int i = 0; i < 8; ++i) x[i] = fix_bits(v8[i], (i < 3 || i == 4 || i == 6) ? wa : ws);
        }
        // contributions as integers (less the kFixMagic each carries); idle lanes give 0
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const unsigned long long xv = x[i] - kFixMagic;
          if (lane >> 5) flp[i * 32 + (lane & 31)] = (long long)xv;
          else acc[i] += xv;
        }
        fold_segment<8, NM>(reinterpret_cast<const long long*>(acc), lane, fl, mine);
      }
      __syncthreads();   // the owner's handed-over contributions are in the partner's scratch
      if (!owner) {
        if (lane < 32) {
#pragma unroll
          for (int i = 0; i < 8; ++i) acc[i] += (unsigned long long)fl[i * 32 + lane];
        }
        __asm__ volatile("" ::: "memory");
        fold_segment<8, NM>(reinterpret_cast<const long long*>(acc), lane, fl, mine);
      }
    } else {
      fold_segment<8, NM>(reinterpret_cast<const long long*>(acc), lane, fl, mine);
    }
  }
  const double snmom = (KIND == 0) ? sn0 : ((KIND <= 2) ? snm : sn1);
  close_row<8, NM>(Scales{a.s1, a.s0, a.p2e1, a.p2e0}, lane, mine, icmom, T, err, (snmom * icmom) * cp,
                   (snmom * icmom) * sp);
}

template <typename ST, int KIND, bool ADAPT = false, bool EXT = false, bool PK = false>
__device__ __forceinline__ void stage3(const StepArgs& a, const StepGeo& G, const ST* X, ST* Xo,
                                       const double (*sJ)[EXT ? 32 : 16], const double* tab, double* snn,
                                       long long gw, long long nw, int lane, long long* fl, I128& T,
                                       int& err, double& emax, const ST* pre = nullptr,
                                       double* gc = nullptr, const double* snp = nullptr,
                                       long long* flp = nullptr, bool owner = false) {
  const Radial g0 = radial_at(a, G.r0), gm = radial_at(a, G.rm), g1 = radial_at(a, G.r1);
  const long long nrow = (long long)a.NS * a.NU * (EXT ? a.NP : 1);
  if constexpr (PK) {   // one row per wavefront
    row3<ST, KIND, false, false, true>(a, X, Xo, gw, G.h, g0, gm, g1, sJ, tab, snn, lane, fl, T, err, emax,
                                       pre, gc, snp, flp, owner);
  } else {
    for (long long row = gw; row < nrow; row += nw)
      row3<ST, KIND, ADAPT, EXT>(a, X, Xo, row, G.h, g0, gm, g1, sJ, tab, snn, lane, fl, T, err, emax,
                                 row == gw ? pre : nullptr, row == gw ? gc : nullptr);
  }
}
// Load the lane's first beam of the wavefront's first row (the next stage starts there),
// so that the load completes while the wavefront waits at the grid barrier.
template <typename ST>
__device__ __forceinline__ void prefetch_first(const StepArgs& a, long long gw, long long nrow, int lane,
                                               ST* pre) {
  if (gw < nrow && lane < a.NE) {
    const ST* X = (const ST*)a.X;
#pragma unroll
    for (int c = 0; c < 6; ++c) pre[c] = X[gw * a.NE + lane + c * a.plane];
  }
}

// ------------------------------------------------------- three flavours, mixed precision
// NB_FP32_STATE: psi stored in FP32 and the per-beam exponentials in FP32; the generators
// come from the FP64 row constants (stages 1-3 rounded to FP32 once per row, the final
// update's Theta summed per beam in FP64 and rounded), the moment contributions, their
// reduction and the renormalisation of the updated state are FP64, and the next moments
// are taken from the rounded stored state.

// One row of the mixed-precision stage with FP32 per-beam arithmetic.
// The moment contributions of a lane's beams (k = lane mod 64 within a segment of 64 x 16
// beams) are summed in FP64 and converted to fixed point once per segment, so the total
// does not depend on the launch shape; 16 contributions below 2^51 each stay below the
// 2^56 that the fold's 64-bit lane sums allow.
// FT: ftab (LDS) holds the vacuum rows and e_k as FP32, eight floats per energy
// (H_ee, H_mumu, H_tautau, H_emu, H_etau, H_mutau, e_k, 0), read by stages 1-3.
template <int KIND, bool FT>
__device__ __forceinline__ void row3m(const StepArgs& a, long long row, const Radial& g0, const Radial& gm,
                                      const Radial& g1, const RowGeo& rg, double icmom, const double (*sJ)[16],
                                      const double* tab, const float* ftab, double* snd, float* snn, int lane,
                                      long long* fl, I128& T, int& err) {
#pragma clang fp contract(fast)
  constexpr int kSeg = 64 * 16;
  const long long plane = a.plane;
  const int NE = a.NE;
  // per-plane bases (uniform) and one 32-bit byte offset per lane: the FP32 planes are
  // below 2^32 bytes (checked at model creation)
  char* Xp[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) Xp[c] = (char*)((float*)a.X + c * plane);
  const int s = (int)(row / a.NU);
  const int an = (s >= (a.NS >> 1)) ? 1 : 0;   // antiparticle row
  // generator row constants (FP64, as in the FP64 stepper): snd[0..8] Q, snd[9..17] P;
  // stages 1-3 use FP32 copies in snn, the final update's Theta is summed in FP64
  double alphaE = 0.0;
  const double alpha = (KIND >= 1)
      ? row_lin3<(KIND >= 1 ? KIND : 1), false, false>(a, an, rg, g0, gm, g1, sJ[0], sJ[1], sJ[2], sJ[3],
                                                        0.0, 0.0, 0.0, 0.0, 0.0, snd, alphaE, lane,
                                                        reinterpret_cast<double*>(fl))
      : 0.0;
  const float alphaf = (float)alpha;
  if (KIND >= 1 && KIND <= 3) {
#pragma unroll
    for (int i = 0; i < 18; ++i) snn[i] = (float)snd[i];
  }
  const double* G = tab + (size_t)(kVacRows3 + s) * NE;
  const long long rb = row * NE;
  I128 mine = i128_zero();
  for (int k0 = lane; k0 - lane < NE; k0 += kSeg) {
    const int kend = min(NE, k0 + kSeg);
    double dacc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    float q[6];
    if (k0 < kend) {
#pragma unroll
      for (int c = 0; c < 6; ++c) q[c] = *(const float*)(Xp[c] + (unsigned)(rb + k0) * 4u);
    }
    for (int k = k0; k < kend; k += 64) {
      cplxf ps[3] = {mkf(q[0], q[1]), mkf(q[2], q[3]), mkf(q[4], q[5])};
      if (k + 64 < kend) {
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = *(const float*)(Xp[c] + (unsigned)(rb + k + 64) * 4u);
      }
      __asm__ volatile("" ::: "memory");
      double pd[6];
      if (KIND >= 1) {
        float v[6], ekf = 0.0f;
        double vd[6];
        if constexpr (KIND <= 3 && FT) {
          const float4 f0 = *reinterpret_cast<const float4*>(ftab + 8 * k);
          const float4 f1 = *reinterpret_cast<const float4*>(ftab + 8 * k + 4);
          v[0] = f0.x; v[1] = f0.y; v[2] = f0.z; v[3] = f0.w; v[4] = f1.x; v[5] = f1.y;
          ekf = f1.z;
        } else {
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            vd[c] = tab[c * NE + k];
            v[c] = (float)vd[c];
          }
          if (KIND == 2) ekf = (float)tab[6 * NE + k];
        }
        if (KIND == 1 || KIND == 3) {
          exp3_apply_f(Herm3f{fmaf(alphaf, v[0], snn[0]), fmaf(alphaf, v[1], snn[1]), fmaf(alphaf, v[2], snn[2]),
                              mkf(fmaf(alphaf, v[3], snn[3]), snn[4]), mkf(fmaf(alphaf, v[4], snn[5]), snn[6]),
                              mkf(fmaf(alphaf, v[5], snn[7]), snn[8])},
                       ps);
        } else if (KIND == 2) {
          const float ek = ekf;
          const float* P = snn + 9;
          exp3_apply_f(Herm3f{fmaf(alphaf, v[0], fmaf(ek, P[0], snn[0])), fmaf(alphaf, v[1], fmaf(ek, P[1], snn[1])),
                              fmaf(alphaf, v[2], fmaf(ek, P[2], snn[2])),
                              mkf(fmaf(alphaf, v[3], fmaf(ek, P[3], snn[3])), fmaf(ek, P[4], snn[4])),
                              mkf(fmaf(alphaf, v[4], fmaf(ek, P[5], snn[5])), fmaf(ek, P[6], snn[6])),
                              mkf(fmaf(alphaf, v[5], fmaf(ek, P[7], snn[7])), fmaf(ek, P[8], snn[8]))},
                       ps);
        } else {
          // Theta = alpha V_k + e_k P + Q.  The generators are nearly constant from step to
          // step (the vacuum term is), so rounding their parts to FP32 would repeat the same
          // phase error every step; Theta is formed in FP64 and rounded once.
          const Herm3 Td = lin3p(alpha, snd + 9, snd, vd, tab[6 * NE + k]);
          const Herm3f Th{(float)Td.d0, (float)Td.d1, (float)Td.d2, mkf((float)Td.o01.re, (float)Td.o01.im),
                          mkf((float)Td.o02.re, (float)Td.o02.im), mkf((float)Td.o12.re, (float)Td.o12.im)};
          // psi + (exp(-i Theta) - 1) psi formed in FP64 from the FP32 increment, then
          // renormalised in FP64, stored rounded to FP32; moments from the stored values
          cplxf dl[3];
          exp3_incr_f(Th, ps, dl);
          const double re0 = (double)ps[0].re + (double)dl[0].re, im0 = (double)ps[0].im + (double)dl[0].im;
          const double re1 = (double)ps[1].re + (double)dl[1].re, im1 = (double)ps[1].im + (double)dl[1].im;
          const double re2 = (double)ps[2].re + (double)dl[2].re, im2 = (double)ps[2].im + (double)dl[2].im;
          const double nrm2 = (fma(re0, re0, im0 * im0) + fma(re1, re1, im1 * im1)) + fma(re2, re2, im2 * im2);
          // 1/sqrt(nrm2) by one Newton step from 1: nrm2 = 1 + d with |d| ~ 1e-7 (a unit
          // FP32-stored state and an increment accurate to FP32), so the error 3 d^2 / 8 is
          // far below FP32 storage precision
          if (a.renorm && !(fabs(nrm2 - 1.0) <= kRenormTol32)) err |= 8;
          const double inv = fma(-0.5, nrm2, 1.5);
          const float o[6] = {(float)(re0 * inv), (float)(im0 * inv), (float)(re1 * inv),
                              (float)(im1 * inv), (float)(re2 * inv), (float)(im2 * inv)};
#pragma unroll
          for (int c = 0; c < 6; ++c) *(float*)(Xp[c] + (unsigned)(rb + k) * 4u) = o[c];
          ps[0] = mkf(o[0], o[1]);
          ps[1] = mkf(o[2], o[3]);
          ps[2] = mkf(o[4], o[5]);
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pd[2 * c] = (double)ps[c].re;
        pd[2 * c + 1] = (double)ps[c].im;
      }
      const cplx p0 = mk(pd[0], pd[1]), p1 = mk(pd[2], pd[3]), p2 = mk(pd[4], pd[5]);
      const double n0 = norm2(p0), nm = norm2(p1), nt = norm2(p2);
      const cplx em = cmul_conjb(p0, p1), et = cmul_conjb(p0, p2), mt = cmul_conjb(p1, p2);
      const double v8[8] = {n0 - nt, nm - nt, em.re, em.im, et.re, et.im, mt.re, mt.im};
      const double w = G[k];
      const double wa = an ? -w : w;   // the negated components of -rho^*
#pragma unroll
      for (int i = 0; i < 8; ++i) dacc[i] = fma((i < 3 || i == 4 || i == 6) ? wa : w, v8[i], dacc[i]);
    }
    long long acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = to_fix(dacc[i], a.s1, kTwo56, err);
    fold_segment<8>(acc, lane, fl, mine);
  }
  close_row<8>(Scales{a.s1, a.s0, a.p2e1, a.p2e0}, lane, mine, icmom, T, err);
}

// Mixed-precision stage: every row with FP32 per-beam arithmetic.  The host runs these
// launches only over steps whose stage generators rotate a beam by at most one radian per
// step (a bound computed from the model's parameters); nearer the neutrinosphere FP32
// cannot hold the per-step phase and the FP64-arithmetic launch on the FP32 state is used.
template <int KIND, bool FT>
__device__ __forceinline__ void stage3m(const StepArgs& a, const StepGeo& G, const double (*sJ)[16],
                                        const double* tab, const float* ftab, double* snn, long long gw,
                                        long long nw, int lane, long long* fl, I128& T, int& err,
                                        double* gc = nullptr) {
  const Radial g0 = radial_at(a, G.r0), gm = radial_at(a, G.rm), g1 = radial_at(a, G.r1);
  const long long nrow = (long long)a.NS * a.NU;
  for (long long row = gw; row < nrow; row += nw) {
    const int s = (int)(row / a.NU);
    const int j = (int)(row - (long long)s * a.NU);
    RowGeo rg;
    double icmom, sn0, snm, sn1;
    stage_geo<KIND, false>(u_of(j, a.NU), G.h, g0, gm, g1, row == gw ? gc : nullptr, rg, icmom, sn0, snm, sn1);
    row3m<KIND, FT>(a, row, g0, gm, g1, rg, icmom, sJ, tab, ftab, snn, (float*)(snn + 32), lane, fl, T, err);
  }
}

// --------------------------------------------------------------- the stepper
// The energy tables (vacuum terms and weights) are staged into LDS once per launch
// when TLDS (they are read by every row).
// EXT: the extended bulb model (azimuthal bins, four moments); FP64 only.
// BS: threads per block (512 or 256; every array and loop bound below is a constant).
// PK: packed row tails (row3); the host launches this variant only when every wavefront of
// the grid owns exactly one row and the row length qualifies.
template <int NF, typename ST, bool TLDS, bool F32, bool EXT, int BS, bool PK = false>
// Register budget: the two-flavour instantiations at 256 threads per block are held to 168
// VGPRs (three wavefronts per SIMD, three blocks per CU); the others keep the compiler's
// choice under the 512-thread bound (two wavefronts per SIMD).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((NF == 2 && BS == 256) ? 3 : 1)))
k_advance(StepArgs a) {
  constexpr int NC = (NF == 2) ? 3 : 8;
  constexpr int NM = EXT ? 4 : 2;
  constexpr int NV = NM * NC;
  constexpr int WPB = BS / 64;
  __shared__ double sJ[4][NV];
  __shared__ I128 sw[WPB][NV];
  __shared__ long long sacc[BS];
  // per wavefront: row constants (mixed: then 32 floats), then the first row's geometry
  __shared__ double snn_all[WPB][F32 ? 64 : 48];
  // the two-flavour extended model's rows fold kFoldRowsExt at a time (group2)
  __shared__ long long sfold[WPB][(NF == 2 && EXT) ? fold2_words(kFoldRowsExt) : (NC + 2) * 64];
  __shared__ double s_sct[kSinCosTab];   // sin/cos constants of the two-flavour rotations
  // extended two-flavour model: each wave's row-constant table
  __shared__ double srt[(NF == 2 && EXT) ? WPB : 1][(NF == 2 && EXT) ? kGroup2 * kRowC : 1];
  extern __shared__ __align__(16) double dyn_tab[];
  // the wavefront index as a wave-uniform (scalar) value: the row indices, their divisions
  // and the row base offsets derived from it then live in scalar registers
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long gw = (long long)blockIdx.x * WPB + wid;
  const long long nw = (long long)gridDim.x * WPB;
  const double* tab = a.tab;
  const float* ftab = nullptr;
  if (launch_aborted(a.sync)) return;
  if (NF == 2 && threadIdx.x == 0) sincos_coefs(s_sct);
  if constexpr (NF == 2) __syncthreads();
  if constexpr (TLDS) {
    const int ntab = ((NF == 2) ? 2 : kVacRows3) * a.NE + a.NS * a.NE;
    for (int i = threadIdx.x; i < ntab; i += BS) dyn_tab[i] = a.tab[i];
    if constexpr (F32) {
      // the FP32 copy of the vacuum rows and e_k, eight floats per energy, after the table
      // (at a 16-byte boundary)
      float* ft = reinterpret_cast<float*>(dyn_tab + ((ntab + 1) & ~1));
      for (int i = threadIdx.x; i < 8 * a.NE; i += BS) {
        const int k = i >> 3, c = i & 7;
        ft[i] = (c < 7) ? (float)a.tab[c * a.NE + k] : 0.0f;
      }
      ftab = ft;
    }
    __syncthreads();
    tab = dyn_tab;
  }
  double* snn = snn_all[wid];
  double* gc = snn + (F32 ? 48 : 32);   // the first row's stage geometry
  long long* fl = sfold[wid];
  const long long step0 = a.step_ctl[0];
  long long nsteps;
  if (a.use_window) {
    // steps [step0, min(target, win_hi)) if step0 lies in the window [win_lo, win_hi)
    nsteps = (step0 < a.win_lo) ? 0LL : max(0LL, min(a.step_ctl[1], a.win_hi) - step0);
  } else {
    nsteps = max(0LL, min(a.nsteps, a.total_steps - step0));
  }
  if (a.use_window && nsteps == 0) return;   // uniform over the grid: nothing to do
  unsigned epoch = 0;
  int err = 0;
  bool ok = true;
  double enone = 0.0;   // error estimate (adaptive runs only)
  I128 T = i128_zero();
  // 3f FP64 arithmetic: each stage's first beam is loaded before the preceding barrier
  ST pre[6] = {};
  const long long nrow3 = (long long)a.NS * a.NU * (EXT ? a.NP : 1);
  if constexpr (PK) {
    // the packed variant's block barriers need one row per wavefront (uniform over the grid):
    // a launch that breaks it ends at once with a range error instead of waiting
    if (!(nrow3 == nw && a.NE > 64 && a.NE <= 64 * 32 && (a.NE & 63) <= 32 && (a.NE & 63) != 0)) {
      if (threadIdx.x == 0)
        __hip_atomic_fetch_or(a.sync + kSyncStatus, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
  // the partner wavefront's constant block and fold scratch (packed tails)
  const double* snp = snn_all[wid ^ (WPB / 2)];
  long long* flp = sfold[wid ^ (WPB / 2)];
  const bool owner = wid < WPB / 2;
  // the stage-1 moments of the current state: left by the previous launch of this variant
  // if it ended at this step (the same values the initial pass would compute), else the
  // initial moment pass
  const long long kind = NF * 16 + (sizeof(ST) == 4 ? 8 : 0) + (F32 ? 4 : 0) + (EXT ? 2 : 0);
  if (a.step_ctl[kCtlMTag] == step0 && a.step_ctl[kCtlMKind] == kind) {
    if constexpr (NF == 3 && !F32) prefetch_first<ST>(a, gw, nrow3, lane, pre);
    if (threadIdx.x < NV) sJ[0][threadIdx.x] = as_double((unsigned long long)a.step_ctl[kCtlMom + threadIdx.x]);
    __syncthreads();
  } else {
    if constexpr (NF == 2) stage2<0, false, EXT>(a, geo_fixed(a, step0), (const double*)a.X, (double*)a.X, sJ, tab, gw, nw, lane, fl, T, err, enone, snn, s_sct, false, srt[EXT ? wid : 0]);
    else if constexpr (F32) stage3m<0, TLDS>(a, geo_fixed(a, step0), sJ, tab, ftab, snn, gw, nw, lane, fl, T, err);
    else { stage3<ST, 0, false, EXT>(a, geo_fixed(a, step0), (const ST*)a.X, (ST*)a.X, sJ, tab, snn, gw, nw, lane, fl, T, err, enone); prefetch_first<ST>(a, gw, nrow3, lane, pre); }
    ok = finish_stage_bs<NV, false, NM, BS>(a, epoch++, T, sw, sacc, sJ[0], 0.0, nullptr, nullptr);
  }
  // the adjoint's forward pass records every stage's moments: [step][slot][NV]
  auto record = [&](long long step, int slot) {
    if (a.Jhist && ok && blockIdx.x == 0 && threadIdx.x < NV)
      a.Jhist[((size_t)step * 4 + slot) * NV + threadIdx.x] = sJ[slot][threadIdx.x];
  };
  record(step0, 0);
  for (long long n = step0; ok && n < step0 + nsteps; ++n) {
    T = i128_zero();
    if constexpr (NF == 2) stage2<1, false, EXT>(a, geo_fixed(a, n), (const double*)a.X, (double*)a.X, sJ, tab, gw, nw, lane, fl, T, err, enone, snn, s_sct, true, srt[EXT ? wid : 0]);
    else if constexpr (F32) stage3m<1, TLDS>(a, geo_fixed(a, n), sJ, tab, ftab, snn, gw, nw, lane, fl, T, err, gc);
    else { stage3<ST, 1, false, EXT, PK>(a, geo_fixed(a, n), (const ST*)a.X, (ST*)a.X, sJ, tab, snn, gw, nw, lane, fl, T, err, enone, pre, gc, snp, flp, owner); prefetch_first<ST>(a, gw, nrow3, lane, pre); }
    if (!(ok = finish_stage_bs<NV, false, NM, BS>(a, epoch++, T, sw, sacc, sJ[1], 0.0, nullptr, nullptr))) break;
    record(n, 1);
    T = i128_zero();
    if constexpr (NF == 2) stage2<2, false, EXT>(a, geo_fixed(a, n), (const double*)a.X, (double*)a.X, sJ, tab, gw, nw, lane, fl, T, err, enone, snn, s_sct, true, srt[EXT ? wid : 0]);
    else if constexpr (F32) stage3m<2, TLDS>(a, geo_fixed(a, n), sJ, tab, ftab, snn, gw, nw, lane, fl, T, err, gc);
    else { stage3<ST, 2, false, EXT, PK>(a, geo_fixed(a, n), (const ST*)a.X, (ST*)a.X, sJ, tab, snn, gw, nw, lane, fl, T, err, enone, pre, gc, snp, flp, owner); prefetch_first<ST>(a, gw, nrow3, lane, pre); }
    if (!(ok = finish_stage_bs<NV, false, NM, BS>(a, epoch++, T, sw, sacc, sJ[2], 0.0, nullptr, nullptr))) break;
    record(n, 2);
    T = i128_zero();
    if constexpr (NF == 2) stage2<3, false, EXT>(a, geo_fixed(a, n), (const double*)a.X, (double*)a.X, sJ, tab, gw, nw, lane, fl, T, err, enone, snn, s_sct, true, srt[EXT ? wid : 0]);
    else if constexpr (F32) stage3m<3, TLDS>(a, geo_fixed(a, n), sJ, tab, ftab, snn, gw, nw, lane, fl, T, err, gc);
    else { stage3<ST, 3, false, EXT, PK>(a, geo_fixed(a, n), (const ST*)a.X, (ST*)a.X, sJ, tab, snn, gw, nw, lane, fl, T, err, enone, pre, gc, snp, flp, owner); prefetch_first<ST>(a, gw, nrow3, lane, pre); }
    if (!(ok = finish_stage_bs<NV, false, NM, BS>(a, epoch++, T, sw, sacc, sJ[3], 0.0, nullptr, nullptr))) break;
    record(n, 3);
    T = i128_zero();
    if constexpr (NF == 2) stage2<4, false, EXT>(a, geo_fixed(a, n), (const double*)a.X, (double*)a.X, sJ, tab, gw, nw, lane, fl, T, err, enone, snn, s_sct, true, srt[EXT ? wid : 0]);
    else if constexpr (F32) stage3m<4, TLDS>(a, geo_fixed(a, n), sJ, tab, ftab, snn, gw, nw, lane, fl, T, err, gc);
    else { stage3<ST, 4, false, EXT, PK>(a, geo_fixed(a, n), (const ST*)a.X, (ST*)a.X, sJ, tab, snn, gw, nw, lane, fl, T, err, enone, pre, gc, snp, flp, owner); prefetch_first<ST>(a, gw, nrow3, lane, pre); }
    ok = finish_stage_bs<NV, false, NM, BS>(a, epoch++, T, sw, sacc, sJ[0], 0.0, nullptr, nullptr);
    record(n + 1, 0);
  }
  if (err) __hip_atomic_fetch_or(a.sync + kSyncStatus, (unsigned)err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // every block read the start step before the first barrier; block 0 passes the last, and
  // leaves the moments of the new state for the next launch
  if (ok && blockIdx.x == 0) {
    if (threadIdx.x < NV) a.step_ctl[kCtlMom + threadIdx.x] = (long long)as_bits(sJ[0][threadIdx.x]);
    if (threadIdx.x == 0) {
      a.step_ctl[0] = step0 + nsteps;
      a.step_ctl[kCtlMTag] = step0 + nsteps;
      a.step_ctl[kCtlMKind] = kind;
    }
  }
}

template __global__ void k_advance<2, double, true, false, false, kBlock>(StepArgs);
template __global__ void k_advance<2, double, false, false, false, kBlock>(StepArgs);
template __global__ void k_advance<3, double, true, false, false, kBlock>(StepArgs);
template __global__ void k_advance<3, double, false, false, false, kBlock>(StepArgs);
template __global__ void k_advance<3, float, true, false, false, kBlock>(StepArgs);
template __global__ void k_advance<3, float, false, false, false, kBlock>(StepArgs);
template __global__ void k_advance<3, float, true, true, false, kBlock>(StepArgs);
template __global__ void k_advance<3, float, false, true, false, kBlock>(StepArgs);
template __global__ void k_advance<2, double, true, false, true, kBlock>(StepArgs);
template __global__ void k_advance<2, double, false, false, true, kBlock>(StepArgs);
template __global__ void k_advance<3, double, true, false, true, kBlock>(StepArgs);
template __global__ void k_advance<3, double, false, false, true, kBlock>(StepArgs);
template __global__ void k_advance<2, double, true, false, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<2, double, false, false, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, double, true, false, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, double, false, false, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, float, true, false, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, float, false, false, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, float, true, true, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, float, false, true, false, kBlockSmall>(StepArgs);
template __global__ void k_advance<2, double, true, false, true, kBlockSmall>(StepArgs);
template __global__ void k_advance<2, double, false, false, true, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, double, true, false, true, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, double, false, false, true, kBlockSmall>(StepArgs);
template __global__ void k_advance<3, double, true, false, false, kBlock, true>(StepArgs);
template __global__ void k_advance<3, double, false, false, false, kBlock, true>(StepArgs);

// --------------------------------------------------------------- adaptive step control
// One persistent launch integrates from r (step_ctl[kCtlR]) with the step length
// step_ctl[kCtlH] to r_end.  Each attempt is a full RKMK4 step from the current state X
// into the other buffer Xn; the final update's barrier also reduces the largest error
// estimate E, from which every block takes the same decision: accept (swap buffers,
// advance r, double h if E <= tol^2/128 and 2h <= h_max) or reject (keep X and the saved
// moments of X, halve h).  The last step is shortened to end at r_end.  At the end each
// wavefront copies its rows back to X if the result sits in the second buffer.
template <int NF, bool TLDS>
__global__ void __launch_bounds__(kBlock) k_adaptive(StepArgs a) {
  constexpr int NC = (NF == 2) ? 3 : 8;
  constexpr int NV = 2 * NC;
  __shared__ double sJ[4][NV];
  __shared__ double sJsave[NV];
  __shared__ double sE[1];
  __shared__ double swm[kBlock / 64];
  __shared__ I128 sw[kBlock / 64][NV];
  __shared__ long long sacc[kBlock];
  __shared__ double snn_all[kBlock / 64][48];   // row constants, then the first row's geometry
  __shared__ long long sfold[kBlock / 64][(NC + 2) * 64];
  __shared__ double s_sct[kSinCosTab];   // sin/cos constants of the two-flavour rotations
  extern __shared__ __align__(16) double dyn_tab[];
  // the wavefront index as a wave-uniform (scalar) value: the row indices, their divisions
  // and the row base offsets derived from it then live in scalar registers
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long gw = (long long)blockIdx.x * (kBlock / 64) + wid;
  const long long nw = (long long)gridDim.x * (kBlock / 64);
  if (launch_aborted(a.sync)) return;
  const double* tab = a.tab;
  if (NF == 2 && threadIdx.x == 0) sincos_coefs(s_sct);
  if constexpr (NF == 2) __syncthreads();
  if constexpr (TLDS) {
    const int ntab = ((NF == 2) ? 2 : kVacRows3) * a.NE + a.NS * a.NE;
    for (int i = threadIdx.x; i < ntab; i += kBlock) dyn_tab[i] = a.tab[i];
    __syncthreads();
    tab = dyn_tab;
  }
  double* snn = snn_all[wid];
  double* gc = snn + 32;   // the first row's stage geometry
  long long* fl = sfold[wid];
  long long* ctl = a.step_ctl;
  double r = as_double((unsigned long long)ctl[kCtlR]);
  double h = as_double((unsigned long long)ctl[kCtlH]);
  double* X = (double*)a.X;
  double* Xn = (double*)a.X2;
  unsigned epoch = 0;
  int err = 0, fail = 0;
  long long nacc = 0, nrej = 0, natt = 0;
  double emax = 0.0;
  I128 T = i128_zero();
  auto stage = [&](auto kind, const StepGeo& G) {
    constexpr int K = decltype(kind)::value;
    if constexpr (NF == 2) stage2<K, K == 4>(a, G, X, Xn, sJ, tab, gw, nw, lane, fl, T, err, emax, snn, s_sct, true);
    else stage3<double, K, K == 4>(a, G, X, Xn, sJ, tab, snn, gw, nw, lane, fl, T, err, emax, nullptr, gc);
  };
  using K0 = std::integral_constant<int, 0>;
  using K1 = std::integral_constant<int, 1>;
  using K2 = std::integral_constant<int, 2>;
  using K3 = std::integral_constant<int, 3>;
  using K4 = std::integral_constant<int, 4>;
  stage(K0{}, StepGeo{r, r, r, 0.0});
  bool ok = finish_stage_bs<NV, false, 2, kBlock>(a, epoch++, T, sw, sacc, sJ[0], 0.0, nullptr, nullptr);
  if (threadIdx.x < NV) sJsave[threadIdx.x] = sJ[0][threadIdx.x];
  while (ok) {
    const bool last = (r + h >= a.r_end);
    const double hs = last ? a.r_end - r : h;
    const StepGeo G{r, r + 0.5 * hs, last ? a.r_end : r + hs, hs};
    T = i128_zero();
    stage(K1{}, G);
    if (!(ok = finish_stage_bs<NV, false, 2, kBlock>(a, epoch++, T, sw, sacc, sJ[1], 0.0, nullptr, nullptr))) break;
    T = i128_zero();
    stage(K2{}, G);
    if (!(ok = finish_stage_bs<NV, false, 2, kBlock>(a, epoch++, T, sw, sacc, sJ[2], 0.0, nullptr, nullptr))) break;
    T = i128_zero();
    stage(K3{}, G);
    if (!(ok = finish_stage_bs<NV, false, 2, kBlock>(a, epoch++, T, sw, sacc, sJ[3], 0.0, nullptr, nullptr))) break;
    T = i128_zero();
    emax = 0.0;
    stage(K4{}, G);
    if (!(ok = finish_stage_bs<NV, true, 2, kBlock>(a, epoch++, T, sw, sacc, sJ[0], emax, swm, sE))) break;
    ++natt;
    const double E = *sE;
    if (E <= a.tol2) {
      ++nacc;
      r = G.r1;
      double* t = X;
      X = Xn;
      Xn = t;
      if (E <= a.tol2 * (1.0 / 128.0) && 2.0 * h <= a.hmax) h = 2.0 * h;
      if (threadIdx.x < NV) sJsave[threadIdx.x] = sJ[0][threadIdx.x];
      if (last) break;
    } else {
      ++nrej;
      h = 0.5 * h;
      if (threadIdx.x < NV) sJ[0][threadIdx.x] = sJsave[threadIdx.x];
      if (h < a.hmin) {
        fail = 1;
        break;
      }
    }
    if (natt >= a.max_attempts) {
      fail = 1;
      break;
    }
    __syncthreads();
  }
  if (ok && X != (double*)a.X) {
    // the accepted state sits in the second buffer: copy this wavefront's rows back
    constexpr int nsc = (NF == 2) ? 3 : 6;
    double* D = (double*)a.X;
    for (long long row = gw; row < (long long)a.NS * a.NU; row += nw)
      for (int k = lane; k < a.NE; k += 64)
#pragma unroll
        for (int c = 0; c < nsc; ++c) D[row * a.NE + k + c * a.plane] = X[row * a.NE + k + c * a.plane];
  }
  if (err) __hip_atomic_fetch_or(a.sync + kSyncStatus, (unsigned)err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (ok && blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[kCtlR] = (long long)as_bits(r);
    ctl[kCtlH] = (long long)as_bits(h);
    ctl[kCtlAcc] = nacc;
    ctl[kCtlRej] = nrej;
    ctl[kCtlAtt] = natt;
    ctl[kCtlFail] = fail;
    ctl[kCtlMTag] = -1;   // the state changed outside the fixed-step launches
    if (!fail) ctl[0] = a.total_steps;
  }
}

template __global__ void k_adaptive<2, true>(StepArgs);
template __global__ void k_adaptive<2, false>(StepArgs);
template __global__ void k_adaptive<3, true>(StepArgs);
template __global__ void k_adaptive<3, false>(StepArgs);

// --------------------------------------------------------------- batched models
// Many independent two-flavour models in one persistent launch (shared step grid).
// Each wavefront owns a contiguous, cost-balanced range of the concatenated rows, so it
// meets only a few models per stage.  Its per-model moment totals are added, as three
// 42-bit limbs, to per-model integer accumulators with device atomics (exact, so the
// result is the same integer as the single-model reduction); a reader rebuilds the
// 128-bit sum from the limbs.  Accumulator sets rotate with the barrier epoch: set e % 6
// collects epoch e, and set (e + 1) % 6 -- last read during epoch e - 1 -- is cleared
// during epoch e.
constexpr unsigned long long kMask42 = (1ull << 42) - 1ull;

__device__ __forceinline__ void acc_add(unsigned long long* slot, const I128& v) {
  const unsigned long long l0 = v.lo & kMask42;
  const unsigned long long l1 = ((v.lo >> 42) | ((unsigned long long)v.hi << 22)) & kMask42;
  const unsigned long long l2 = (unsigned long long)(v.hi >> 20);
  __hip_atomic_fetch_add(slot + 0, l0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(slot + 1, l1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(slot + 2, l2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ I128 acc_read(const unsigned long long* slot) {
  const unsigned long long s0 = __hip_atomic_load(slot + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long s1 = __hip_atomic_load(slot + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const long long s2 = (long long)__hip_atomic_load(slot + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  I128 t = I128{s0, 0ll};
  t = i128_add(t, I128{s1 << 42, (long long)(s1 >> 22)});
  t = i128_add(t, I128{0ull, s2 << 20});
  return t;
}
__device__ __forceinline__ unsigned long long* acc_slot(const BatchArgs& a, unsigned epoch, int m) {
  return a.acc + ((size_t)(epoch % kAccSets) * a.nmodels + m) * 6 * kAccLimbs;
}

// Flags-only grid barrier (the sums are already in the accumulators, added with
// agent-scope atomics before the workgroup barrier inside the arrival).
__device__ bool grid_barrier(const BatchArgs& a, unsigned epoch) {
  const unsigned want = epoch + 1u;
  if (blockIdx.x != 0) return arrive_and_wait(a.sync, a.cancel, a.timeout_ticks, want);
  if (!wait_arrivals(a.sync, a.cancel, a.timeout_ticks, want)) return false;
  release_grid(a.sync, want);
  return true;
}

// Rows are taken in groups of up to kGroup rows of one model: lane l first computes the
// constants of the group's row l (row_setup2, the arithmetic every lane of the row would
// otherwise repeat) into the wave's table rt, then the rows run one after the other.
constexpr int kGroup = 16;
template <int KIND>
__device__ void batch_stage(const BatchArgs& a, long long n, unsigned epoch, long long r0w,
                            long long r1w, int lane, double (*Jv)[6], long long* fl, double* cb,
                            double* rt, const double* sct, int& err) {
  const double r0 = a.rs + (double)n * a.h;
  const double rm = r0 + 0.5 * a.h;
  const double r1 = a.rs + (double)(n + 1) * a.h;
  // epoch of the slot holding J^(i+1) of this step: epoch - KIND + i
  int m = -1;
  long long mrow0 = 0, mrow1 = 0, mbeam0 = 0, mtab0 = 0;
  int mNE = 0, mNU = 1;
  const double* J[4] = {Jv[0], Jv[1], Jv[2], Jv[3]};   // this wave's LDS block
  I128 T = i128_zero();
  for (long long row = r0w; row < r1w;) {
    if (m < 0 || row >= mrow1) {
      if (m >= 0 && lane < 6) acc_add(acc_slot(a, epoch, m) + lane * kAccLimbs, T);
      T = i128_zero();
      if (m < 0) {                      // first model of the range: binary search
        int lo = 0, hi = a.nmodels - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (a.models[mid].row0 <= row) lo = mid; else hi = mid - 1;
        }
        m = lo;
      } else {
        while (row >= a.models[m].row0 + 2LL * a.models[m].NU) ++m;
      }
      const BatchModel* md = a.models + m;
      mrow0 = md->row0;
      mNE = md->NE;
      mNU = md->NU;
      mrow1 = mrow0 + 2LL * mNU;
      mbeam0 = md->beam0;
      mtab0 = md->tab0;
      const double lam0 = md->lam0;
      const Scales sc{md->s1, md->s0, md->p2e1, md->p2e0};
      put_stage2(cb, lane, radial(a.R, a.ne_power, lam0, r0), radial(a.R, a.ne_power, lam0, rm),
                 radial(a.R, a.ne_power, lam0, r1), sc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool need = (i == 0) ? (KIND == 1 || KIND == 2 || KIND == 4)
                                   : (i == 1 ? (KIND == 2 || KIND == 4) : (i == 2 ? KIND >= 3 : KIND == 4));
        if (!need) continue;
        const unsigned long long* sl = acc_slot(a, epoch - (unsigned)KIND + (unsigned)i, m);
#pragma unroll
        for (int v = 0; v < 6; ++v)
          Jv[i][v] = i128_to_double(acc_read(sl + v * kAccLimbs)) * (v < 3 ? sc.p2e0 : sc.p2e1);
      }
    }
    const long long gend = min(min(r1w, mrow1), row + (long long)kGroup);
    const int gn = (int)(gend - row);
    __asm__ volatile("" ::: "memory");   // the previous group's rows have read their blocks
    if (lane < gn) {
      const int lr = (int)(row + lane - mrow0);
      const int s = lr / mNU;
      const int j = lr - s * mNU;
      row_setup2<KIND, false>(u_of(j, mNU), a.h, cb, J, 0.0, 0.0, nullptr, true, rt + lane * kRowC);
      rt[lane * kRowC + kRowS] = (double)s;
      rt[lane * kRowC + kRowA] = (double)s;   // two tracked species: row s is anti iff s = 1
    }
    __asm__ volatile("" ::: "memory");
    if (mNE <= kGroupMaxNE) {
      group2<KIND, false, kFoldRowsBatch>(a.X, a.plane, mbeam0 + (row - mrow0) * mNE, mNE, gn, a.tab + mtab0, cb, rt,
                          a.renorm, lane, fl, T, err, sct);
      row += gn;
    } else {
      for (int i = 0; i < gn; ++i, ++row) {
        const long long lr = row - mrow0;
        const int s = (int)(lr / mNU);
        double enone = 0.0;
        row2<KIND, false, false, true>(a.X, a.X, a.plane, mbeam0 + lr * mNE, mNE, s, 0.0, a.h, a.tab + mtab0,
                                       cb, J, a.renorm, lane, fl, T, err, enone, 0.0, 0.0, -1, false, sct,
                                       rt + i * kRowC);
      }
    }
  }
  if (m >= 0 && lane < 6) acc_add(acc_slot(a, epoch, m) + lane * kAccLimbs, T);
  // clear the set the next epoch will collect into
  if (blockIdx.x == 0) {
    unsigned long long* z = a.acc + (size_t)((epoch + 1u) % kAccSets) * a.nmodels * 6 * kAccLimbs;
    for (int i = threadIdx.x; i < a.nmodels * 6 * kAccLimbs; i += blockDim.x)
      __hip_atomic_store(z + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Four wavefronts per SIMD (128 VGPRs; the row groups' set-up spills about 230 bytes per
// lane, outside the chunk loop): the rows of a batch are short (50-400 energies), so a wave
// spends much of its time on row set-up and the first load of each row, which more
// wavefronts hide.  Measured on the 256-model batch: 4.35 (two wavefronts per SIMD) -> 4.20
// (four, 512 threads, 224-byte spill) -> 3.52 (three, 256 threads) -> 3.19 ms per step
// (four, 256 threads, with the wavefront index scalar); with the lane-parallel row groups,
// the chunks streamed across rows and the table prefetch 2.53 ms (three wavefronts per SIMD
// then measure 2.65).
template <int BS>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_batch2(BatchArgs a) {
  __shared__ double sJw[BS / 64][4][6];
  // (fold2_words(R) also covers row2's fold_segment<3>: 3 * 64 + 63 words)
  __shared__ long long sfold[BS / 64][fold2_words(kFoldRowsBatch)];
  __shared__ double scb[BS / 64][kC2Size];
  __shared__ double srt[BS / 64][kGroup * kRowC];   // each wave's row-constant table
  __shared__ double s_sct[kSinCosTab];   // sin/cos constants of the rotations
  if (launch_aborted(a.sync)) return;
  if (threadIdx.x == 0) sincos_coefs(s_sct);
  __syncthreads();
  // the wavefront index as a wave-uniform (scalar) value: the row indices, their divisions
  // and the row base offsets derived from it then live in scalar registers
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double (*Jv)[6] = sJw[wid];
  const long long w = (long long)blockIdx.x * (BS / 64) + wid;
  const long long r0w = min(max(a.wave_row0[w], 0LL), a.total_rows);
  const long long r1w = min(max(a.wave_row0[w + 1], r0w), a.total_rows);
  const long long step0 = *a.step_ctl;
  const long long nsteps = max(0LL, min(a.nsteps, a.total_steps - step0));
  unsigned epoch = 0;
  int err = 0;
  bool ok;
  batch_stage<0>(a, step0, epoch, r0w, r1w, lane, Jv, sfold[wid], scb[wid], srt[wid], s_sct, err);
  ok = grid_barrier(a, epoch++);
  for (long long n = step0; ok && n < step0 + nsteps; ++n) {
    batch_stage<1>(a, n, epoch, r0w, r1w, lane, Jv, sfold[wid], scb[wid], srt[wid], s_sct, err);
    if (!(ok = grid_barrier(a, epoch++))) break;
    batch_stage<2>(a, n, epoch, r0w, r1w, lane, Jv, sfold[wid], scb[wid], srt[wid], s_sct, err);
    if (!(ok = grid_barrier(a, epoch++))) break;
    batch_stage<3>(a, n, epoch, r0w, r1w, lane, Jv, sfold[wid], scb[wid], srt[wid], s_sct, err);
    if (!(ok = grid_barrier(a, epoch++))) break;
    batch_stage<4>(a, n, epoch, r0w, r1w, lane, Jv, sfold[wid], scb[wid], srt[wid], s_sct, err);
    ok = grid_barrier(a, epoch++);
  }
  if (err) __hip_atomic_fetch_or(a.sync + kSyncStatus, (unsigned)err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (ok && blockIdx.x == 0 && threadIdx.x == 0) *a.step_ctl = step0 + nsteps;
}
template __global__ void k_batch2<kBlock>(BatchArgs);
template __global__ void k_batch2<kBlockSmall>(BatchArgs);

// ----------------------------------------------------------------- small kernels
__global__ void k_zero_u64(unsigned long long* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}
// The state was set or reset: the step, and no moments left for the next launch.
__global__ void k_set_step(long long* step_ctl, long long step) {
  step_ctl[0] = step;
  step_ctl[kCtlMTag] = -1;
}
// The status word and the device step counter into host memory (one small write the host
// reads after synchronising, instead of two copies).
__global__ void k_status_out(const unsigned int* sync, const long long* step_ctl, long long* host) {
  __hip_atomic_store(host, (long long)sync[kSyncStatus], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(host + 1, step_ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Target of a group of windowed launches: k more steps from the device step counter.
__global__ void k_set_target(long long* step_ctl, long long k, long long total) {
  step_ctl[1] = min(step_ctl[0] + k, total);
}

// Clear the barrier and reduction words before a persistent launch (keep_status: keep the
// status bits of earlier launches of the same call).  If the host has set the model's
// cancel word (fine-grained host memory; nullptr: none), the abort word is set instead of
// cleared, with status bit 2, so that the next persistent launch returns at once.
__global__ void k_zero_sync(unsigned int* sync, int keep_status, const unsigned* cancel) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kSyncWords; i += gridDim.x * blockDim.x) {
    if (i == kSyncStatus) continue;   // written with the abort word
    if (i == kSyncAbort) {
      const unsigned c =
          cancel ? __hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0u;
      const unsigned st = keep_status ? sync[kSyncStatus] : 0u;
      sync[kSyncAbort] = c ? 1u : 0u;
      sync[kSyncStatus] = st | (c ? 4u : 0u);
      continue;
    }
    sync[i] = 0u;
  }
}

// Initial flavour eigenstates (Sec. 3.4): species row s = b / per_species is born in
// flavour s % nfl (nfl = 1 when only electron-born beams are tracked); 2f: P = (0, 0, +-1),
// 3f: psi = the unit vector of that flavour.
template <typename ST>
__global__ void k_init(ST* X, long long nb, long long plane, int nsc, long long per_species, int nfl) {
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int fl = (int)((b / per_species) % nfl);
  for (int c = 0; c < nsc; ++c) {
    ST v = (ST)0;
    if (nsc == 3) v = (c == 2) ? (ST)(fl == 0 ? 1 : -1) : (ST)0;
    else v = (c == 2 * fl) ? (ST)1 : (ST)0;
    X[b + c * plane] = v;
  }
}
template __global__ void k_init<double>(double*, long long, long long, int, long long, int);
template __global__ void k_init<float>(float*, long long, long long, int, long long, int);

template <typename ST>
__global__ void k_read_pee(const ST* X, long long nb, long long plane, int nsc, double* out) {
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  if (nsc == 3) {
    out[b] = 0.5 * (1.0 + (double)X[b + 2 * plane]);
  } else {
    const double re = (double)X[b], im = (double)X[b + plane];
    out[b] = fma(re, re, im * im);
  }
}
template __global__ void k_read_pee<double>(const double*, long long, long long, int, double*);
template __global__ void k_read_pee<float>(const float*, long long, long long, int, double*);

// State exchange with FP64 [comp][beam] planes (dir 0: state -> out, 1: in -> state).
template <typename ST>
__global__ void k_state_xfer(ST* X, long long nb, long long plane, int nsc, double* buf, int dir) {
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  for (int c = 0; c < nsc; ++c) {
    if (dir == 0) buf[c * nb + b] = (double)X[b + c * plane];
    else X[b + c * plane] = (ST)buf[c * nb + b];
  }
}
template __global__ void k_state_xfer<double>(double*, long long, long long, int, double*, int);
template __global__ void k_state_xfer<float>(float*, long long, long long, int, double*, int);

}  // namespace nb
