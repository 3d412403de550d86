// nb_stage.h -- device helpers shared by the stepping kernels and the adjoint kernel:
// radial profiles, emission-bin geometry, the nu-nu term of a row, the two-flavour stage
// generator and the time-limited barrier wait.
#pragma once
#include "nb_device.h"
#include "nb_internal.h"

namespace nb {

struct Radial {
  double q2, lam, mu, qp;  // (R/r)^2, sqrt2 G_F n_e(r), R^2/2r^2, (R/r)^ne_power
};

__device__ __forceinline__ Radial radial(double R, int ne_power, double lam0, double r) {
  Radial g;
  const double q = R / r;
  g.q2 = q * q;
  double qp = 1.0;
  for (int i = 0; i < ne_power; ++i) qp = qp * q;
  g.lam = lam0 * qp;     // sqrt2 G_F n_e(r)
  g.mu = 0.5 * g.q2;     // R^2 / 2r^2 from d cos(theta') = (R^2/2r^2) du / cos(theta')
  g.qp = qp;
  return g;
}
__device__ __forceinline__ double as_double(unsigned long long u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ unsigned long long as_bits(double d) { return (unsigned long long)__double_as_longlong(d); }

// Grid barriers.  Within one launch a beam's state is touched only by the wavefront that
// owns its row, so the only data that crosses blocks are the block partials, the reduced
// moments and the barrier words -- and every one of those is written and read with
// agent-scope atomics, which are coherent at the device level without L2 write-back or
// invalidation.  Ordering comes from the protocol itself: a block's partial stores
// complete before its arrival word is stored (the workgroup barrier in between waits for
// all of the block's outstanding memory operations), and a waiter issues its loads of the
// published data only after it has read the word that announces them.  So the barrier
// needs no cache maintenance at all: the state written in the same stage stays in L2.

// Checked every 32nd poll (it) of a wait: true if another block has aborted, or if this
// wait, begun at t0, has passed the launch's time limit (then it sets the abort word and
// status bit 1 so that every other waiter gives up too), or -- every 1024th poll -- if the
// host has set the model's cancel word, a word of fine-grained host memory (then it sets
// the abort word and status bit 2).
__device__ __forceinline__ bool give_up(unsigned* sync, const unsigned* cancel, unsigned long long t0,
                                        unsigned long long timeout_ticks, unsigned it) {
  if (__hip_atomic_load(sync + kSyncAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
  unsigned bit = 0u;
  if (wall_clock64() - t0 > timeout_ticks) bit = 2u;
  else if (cancel && (it & 1023u) == 0u &&
           __hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
    bit = 4u;
  if (!bit) return false;
  __hip_atomic_store(sync + kSyncAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_or(sync + kSyncStatus, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}
// Read at the start of a persistent launch (all threads of the block call this; thread 0
// reads, the block shares its answer): the abort word, set before the launch by the
// sync-word clear when the host had cancelled the model (every block then returns at once,
// leaving the state as it was), or during it by a block that gave up.
__device__ __forceinline__ bool launch_aborted(const unsigned* sync) {
  return __syncthreads_or(threadIdx.x == 0 &&
                          __hip_atomic_load(sync + kSyncAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u);
}

// Poll *w (relaxed) until it reaches want; gives up when another block has aborted or the
// launch's time limit passes (then it sets the abort word and status bit 1).  The abort
// word and the clock are read only every 32nd poll, so a poll costs one load round trip.
__device__ __forceinline__ bool poll_until(unsigned* sync, const unsigned* cancel,
                                           unsigned long long timeout_ticks, unsigned* w, unsigned want) {
  const unsigned long long t0 = wall_clock64();
  for (unsigned it = 1;; ++it) {
    if (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) return true;
    if ((it & 31u) == 0u && give_up(sync, cancel, t0, timeout_ticks, it)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}
// Block 0 of a barrier (all its threads call this): the first wavefront polls every other
// block's arrival word, all of a lane's words per round so that their loads overlap.
// Returns false on give-up.
__device__ __forceinline__ bool wait_arrivals(unsigned* sync, const unsigned* cancel,
                                              unsigned long long timeout_ticks, unsigned want) {
  int ok = 1;
  if (threadIdx.x < 64) {
    const unsigned long long t0 = wall_clock64();
    for (unsigned it = 1;; ++it) {
      unsigned lowest = 0xffffffffu;
      for (unsigned b = 1 + threadIdx.x; b < gridDim.x; b += 64)
        lowest = min(lowest, __hip_atomic_load(sync + kSyncArrive + b * kLineWords, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT));
      if (lowest >= want) break;
      if ((it & 31u) == 0u && give_up(sync, cancel, t0, timeout_ticks, it)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return !__syncthreads_or(!ok);
}
// A non-zero block arrives (all its threads call this, after their partial stores) and
// waits for block 0's release flag.  Returns false on give-up.
__device__ __forceinline__ bool arrive_and_wait(unsigned* sync, const unsigned* cancel,
                                                unsigned long long timeout_ticks, unsigned want) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(sync + kSyncArrive + blockIdx.x * kLineWords, want, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    s_ok = poll_until(sync, cancel, timeout_ticks, sync + kSyncFlag + (blockIdx.x % kFlagCopies) * kLineWords,
                      want) ? 1 : 0;
  }
  __syncthreads();
  return s_ok != 0;
}
// Block 0 releases the grid (all its threads call this, after their result stores).
__device__ __forceinline__ void release_grid(unsigned* sync, unsigned want) {
  __syncthreads();
  if (threadIdx.x < kFlagCopies)
    __hip_atomic_store(sync + kSyncFlag + threadIdx.x * kLineWords, want, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Geometry of one emission bin u at the three stage radii of a step.
struct RowGeo {
  double c0, cm, c1, hc0, hcm, hc1;
};
__device__ __forceinline__ RowGeo row_geo(double u, double h, const Radial& g0, const Radial& gm,
                                          const Radial& g1) {
  RowGeo r;
  r.c0 = sqrt(1.0 - u * g0.q2);
  r.cm = sqrt(1.0 - u * gm.q2);
  r.c1 = sqrt(1.0 - u * g1.q2);
  r.hc0 = h / r.c0;
  r.hcm = h / r.cm;
  r.hc1 = h / r.c1;
  return r;
}
__device__ __forceinline__ double u_of(int j, int NU) { return ((double)j + 0.5) / (double)NU; }
// The neutrino-neutrino term mu (J0 - c J1) of a row: the same for every energy bin.
template <int NC>
__device__ __forceinline__ void nunu(const double* J, double mu, double c, double* nn) {
#pragma unroll
  for (int i = 0; i < NC; ++i) nn[i] = mu * (J[i] - c * J[NC + i]);
}
// Extended bulb model: the azimuthal part of 1 - v.v' adds - sin(theta) (cos(phi) J_sc +
// sin(phi) J_ss); J = [J0 | J1 | J_sc | J_ss].  The same for every energy bin of the row.
template <int NC>
__device__ __forceinline__ void nunu_ext(const double* J, double mu, double c, double sn, double cp,
                                         double sp, double* nn) {
#pragma unroll
  for (int i = 0; i < NC; ++i)
    nn[i] = mu * ((J[i] - c * J[NC + i]) - sn * (cp * J[2 * NC + i] + sp * J[3 * NC + i]));
}
// Row nn terms of either model (EXT: the extended bulb model).
template <int NC, bool EXT>
__device__ __forceinline__ void nunu_row(const double* J, double mu, double c, double sn, double cp,
                                         double sp, double* nn) {
  if constexpr (EXT) nunu_ext<NC>(J, mu, c, sn, cp, sp, nn);
  else nunu<NC>(J, mu, c, nn);
}
// ----------------------------------------------------------------- two flavours
// Stage generator f = (h/c) B of beam (s, k) with B = B_vac + lam e_z + nn for
// neutrinos and B_vac - lam e_z - nn^* (nn^* = (x, -y, z)) for antineutrinos.
__device__ __forceinline__ void gen2(int s, double bx, double bz, double lam, const double* nn,
                                     double hc, double f[3]) {
  double B0, B1, B2;
  if (s == 0) {
    B0 = bx + nn[0];
    B1 = nn[1];
    B2 = (bz + lam) + nn[2];
  } else {
    B0 = bx - nn[0];
    B1 = nn[1];
    B2 = (bz - lam) - nn[2];
  }
  f[0] = hc * B0;
  f[1] = hc * B1;
  f[2] = hc * B2;
}


}  // namespace nb
