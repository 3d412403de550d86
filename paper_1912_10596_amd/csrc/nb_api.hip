// nb_api.hip -- host runtime behind include/nubulb.h: parameter validation, host tables,
// workspace layout, persistent launches, status checks, the autotuner and its cache.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/nubulb.h"
#include "nb_internal.h"

namespace nb {
template <int NF, typename ST, bool TLDS, bool F32, bool EXT, int BS, bool PK>
__global__ void k_advance(StepArgs a);
template <int BS>
__global__ void k_batch2(BatchArgs a);
template <int BPT>
__global__ void k_adjoint2(AdjArgs a);
template <int NF, bool TLDS>
__global__ void k_adaptive(StepArgs a);
__global__ void k_zero_sync(unsigned int* sync, int keep_status, const unsigned* cancel);
__global__ void k_zero_u64(unsigned long long* p, long long n);
__global__ void k_set_step(long long* step_ctl, long long step);
__global__ void k_status_out(const unsigned int* sync, const long long* step_ctl, long long* host);
__global__ void k_set_target(long long* step_ctl, long long k, long long total);
template <typename ST>
__global__ void k_init(ST* X, long long nb, long long plane, int nsc, long long per_species, int nfl);
template <typename ST>
__global__ void k_read_pee(const ST* X, long long nb, long long plane, int nsc, double* out);
template <typename ST>
__global__ void k_state_xfer(ST* X, long long nb, long long plane, int nsc, double* buf, int dir);
}  // namespace nb

using namespace nb;

// ------------------------------------------------------------------- errors
static thread_local std::string g_err;
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
#define NB_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return fail(NB_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* nb_last_error(void) { return g_err.c_str(); }

// --------------------------------------------------------------- cancel words
// Every bound model owns one 32-bit word of fine-grained (coherent) pinned host memory:
// nb_cancel writes it from any host thread, the sync-word clear before each persistent
// launch reads it, and waiting blocks poll it.  Words come from pages allocated once per
// process and never freed (a freed model's word is reused).
constexpr int kCancelPage = 1024;
static std::mutex g_cancel_mu;
static std::vector<unsigned*> g_cancel_free;
static int cancel_word_take(unsigned** host, const unsigned** dev) {
  std::lock_guard<std::mutex> lock(g_cancel_mu);
  if (g_cancel_free.empty()) {
    void* page = nullptr;
    NB_HIP(hipHostMalloc(&page, sizeof(unsigned) * kCancelPage,
                         hipHostMallocPortable | hipHostMallocMapped | hipHostMallocCoherent));
    unsigned* w = (unsigned*)page;
    for (int i = kCancelPage - 1; i >= 0; --i) {
      w[i] = 0u;
      g_cancel_free.push_back(w + i);
    }
  }
  unsigned* w = g_cancel_free.back();
  void* d = nullptr;
  NB_HIP(hipHostGetDevicePointer(&d, w, 0));
  g_cancel_free.pop_back();
  __atomic_store_n(w, 0u, __ATOMIC_SEQ_CST);
  *host = w;
  *dev = (const unsigned*)d;
  return NB_OK;
}
static void cancel_word_give(unsigned* w) {
  if (!w) return;
  std::lock_guard<std::mutex> lock(g_cancel_mu);
  __atomic_store_n(w, 0u, __ATOMIC_SEQ_CST);
  g_cancel_free.push_back(w);
}

// --------------------------------------------------------------- constants
// sqrt(2) G_F (hbar c)^3 in km^-1 cm^3 with G_F = 1.1663787e-5 GeV^-2 and
// hbar c = 1.973269804e-14 GeV cm = 1.973269804e-19 GeV km.
static double potential_per_density() {
  const double hc_cm = 1.973269804e-14, hc_km = 1.973269804e-19;
  return (1.4142135623730951 * 1.1663787e-5) * ((hc_cm * hc_cm) * hc_cm) / hc_km;
}
static constexpr double kVac = 1.0 / (4.0e6 * 1.973269804e-10);  // dm^2/(4E): eV^2/MeV -> km^-1
static constexpr double kErgMeV = 624150.9074460763;
static constexpr double kClight = 2.99792458e10;                  // cm/s
static constexpr double kPi = 3.141592653589793;
static constexpr double kFD2 = 1.8030853547393914;                // int x^2/(e^x+1) dx
static constexpr double kFD3 = 5.682196976983475;                 // int x^3/(e^x+1) dx

static double fd_spectrum(double E, double T) {  // normalised Fermi-Dirac, zero potential
  return (E * E) / ((kFD2 * ((T * T) * T)) * (std::exp(E / T) + 1.0));
}

// ---------------------------------------------------------------- the model
// One model (or, for a batch, one member): parameters and host tables.
struct Sub {
  nb_params p{};
  long long NE = 0, NU = 0, NP = 1, beam0 = 0, row0 = 0, tab0 = 0;  // NP: azimuthal bins
  int NS = 2;                        // species rows: 2, or 2 n_flavor when every flavour is tracked
  double h = 0, lam0 = 0, kappa0 = 0, s1 = 0, s0 = 0, p2e1 = 0, p2e0 = 0;
  double vac_max = 0;                // max over energy bins of sum |H_vac entries|
  double v0[6] = {0, 0, 0, 0, 0, 0};  // 3f: vacuum Hamiltonian times E (bin k: v0 / E_k)
  long long fp32_from = 0;           // mixed precision: first step run with FP32 arithmetic
  int e1 = 0, e0 = 0, nf = 2;
  std::vector<double> E, tab;
  std::vector<double> dtab;          // 2f: [dG0/dL_e | dG1/dL_ebar | dG/dL_x | dbx/dth | dbz/dth] x NE
};

struct nb_model {
  nb_params p{};                     // the (first) model's parameters; the shared step grid
  int nf = 2, nc = 3, nsc = 3, nmodels = 1;
  bool batch = false;
  long long nb = 0, plane = 0, rows = 0;
  std::vector<Sub> subs;
  std::vector<double> tab;           // concatenated device table image
  long long step = 0;
  // launch shape of the fixed-step kernels (autotuner results or nb_set_tuning): threads per
  // block, block cap and the per-row overhead of the batch partition's cost model
  int bs = kBlock;
  bool tuned = false;                // bs / tune_blocks / tune_row_cost set by the autotuner or the caller
  int tune_blocks = 0;
  double tune_row_cost = 1.0;
  // bound state
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0, cus = 0, nblocks = 0;
  int cap512 = 0, cap256 = 0;        // resident blocks of the fixed-step kernels at 512 / 256 threads
  int cap_adaptive = 0;              // resident blocks of the adaptive kernel (512 threads)
  unsigned* cancel = nullptr;        // this model's cancel word (fine-grained host memory)
  const unsigned* cancel_dev = nullptr;  // its device address
  unsigned long long ticks_per_s = 0;
  size_t off_X = 0, off_tab = 0, off_sync = 0, off_ctl = 0;
  size_t off_models = 0, off_waves = 0, off_acc = 0, need = 0;
  size_t off_adj = 0, off_spill = 0, off_jhist = 0, off_dtab = 0, off_aout = 0, off_X2 = 0;
  double* jhist = nullptr;           // set while the adjoint's forward pass records moments
  int adj_blocks = 0, adj_bpt = 0;
  long long* pinned = nullptr;       // [0] status, [1] step, [8..12] adjoint gradients
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  long long graph_steps = 0;
  int graph_bs = 0, graph_blocks = 0;   // launch shape recorded in the graph
  // set only inside nb_step_static: barrier words and batch accumulators taken from the
  // static scratch array instead of the workspace
  unsigned int* sync_static = nullptr;
  unsigned long long* acc_static = nullptr;
};

// Barrier and reduction words, and batch moment accumulators, of the stepping launches.
static unsigned int* sync_words(const nb_model* m) {
  return m->sync_static ? m->sync_static : (unsigned int*)(m->ws + m->off_sync);
}
static unsigned long long* acc_words(const nb_model* m) {
  return m->acc_static ? m->acc_static : (unsigned long long*)(m->ws + m->off_acc);
}

static bool state_fp32(const nb_model* m) { return m->nf == 3 && m->p.precision == NB_FP32_STATE; }

static int validate(const nb_params* p) {
  if (!p) return fail(NB_EINVAL, "params is NULL");
  if (p->n_flavor != 2 && p->n_flavor != 3) return fail(NB_EINVAL, "n_flavor must be 2 or 3");
  if (p->n_energy < 1 || p->n_u < 1) return fail(NB_EINVAL, "n_energy and n_u must be >= 1");
  if ((long long)p->n_energy * p->n_u > (1LL << 34)) return fail(NB_EINVAL, "too many beams");
  if (p->n_steps < 1) return fail(NB_EINVAL, "n_steps must be >= 1");
  if (!(p->r_nu_km > 0.0) || !(p->r_start_km >= p->r_nu_km) || !(p->r_end_km > p->r_start_km))
    return fail(NB_EINVAL, "need 0 < r_nu <= r_start < r_end");
  if (!(p->e_min_mev > 0.0) || !(p->e_max_mev > p->e_min_mev))
    return fail(NB_EINVAL, "need 0 < e_min < e_max");
  if (p->delta_cp != 0.0) return fail(NB_EINVAL, "delta_cp must be 0");
  if (p->ne_power < 0 || p->ne_power > 8) return fail(NB_EINVAL, "ne_power must be in 0..8");
  if (p->precision != NB_FP64 && p->precision != NB_FP32_STATE)
    return fail(NB_EINVAL, "unknown precision");
  if (p->precision == NB_FP32_STATE && p->n_flavor != 3)
    return fail(NB_EINVAL, "FP32 state is a three-flavour mode");
  // the FP32 stepping kernel addresses a state plane with 32-bit byte offsets
  if (p->precision == NB_FP32_STATE &&
      (long long)p->n_energy * p->n_u * (p->track_all ? 2 * p->n_flavor : 2) > (1LL << 30) - 64)
    return fail(NB_EINVAL, "FP32 state planes must stay below 4 GiB (at most 2^30 - 64 beams)");
  for (int i = 0; i < 3; ++i)
    if (!(p->temp_mev[i] > 0.0) || !(p->lum_erg_s[i] >= 0.0))
      return fail(NB_EINVAL, "temperatures must be > 0 and luminosities >= 0");
  if (!(std::isfinite(p->n0_cm3) && p->n0_cm3 >= 0.0)) return fail(NB_EINVAL, "n0 must be >= 0");
  if (p->adjoint_ckpt < 0) return fail(NB_EINVAL, "adjoint_ckpt must be >= 0");
  if (p->adjoint_ckpt > 0 && (p->n_flavor != 2 || p->precision != NB_FP64))
    return fail(NB_EINVAL, "the adjoint is a two-flavour FP64 mode");
  if (p->max_blocks < 0) return fail(NB_EINVAL, "max_blocks must be >= 0");
  if (p->adaptive != 0 && p->adaptive != 1) return fail(NB_EINVAL, "adaptive must be 0 or 1");
  if (p->adaptive && p->precision != NB_FP64) return fail(NB_EINVAL, "adaptive stepping is an FP64 mode");
  if (p->n_phi < 0 || p->n_phi > 4096) return fail(NB_EINVAL, "n_phi must be in 0..4096");
  if (p->track_all != 0 && p->track_all != 1) return fail(NB_EINVAL, "track_all must be 0 or 1");
  if (p->reserved != 0) return fail(NB_EINVAL, "reserved must be 0");
  if (p->temp_xbar_mev != 0.0 && (!(p->temp_xbar_mev > 0.0) || !(p->lum_xbar_erg_s >= 0.0)))
    return fail(NB_EINVAL, "anti-nu_x temperature must be > 0 (or 0) and luminosity >= 0");
  if (p->adjoint_ckpt > 0 && (p->track_all || p->temp_xbar_mev != 0.0))
    return fail(NB_EINVAL, "the adjoint takes anti-nu_x = nu_x and two tracked species");
  if (p->n_phi > 0 && (p->precision != NB_FP64 || p->adjoint_ckpt != 0 || p->adaptive != 0))
    return fail(NB_EINVAL, "the extended bulb model is an FP64 fixed-step mode without adjoint");
  if ((long long)p->n_energy * p->n_u * (p->n_phi > 0 ? p->n_phi : 1) *
          (p->track_all ? p->n_flavor : 1) > (1LL << 34))
    return fail(NB_EINVAL, "too many beams");
  return NB_OK;
}

// Host tables of one model (Sec. 2 / Sec. 3.2): bin midpoints, Fermi-Dirac spectra,
// number luminosities N = L/<E>, weights g = kappa0 du dE (N_a f_a - N_x f_x), vacuum
// Hamiltonians per energy, fixed-point scales.
static void build_tables(Sub* m) {
  const nb_params& p = m->p;
  const long long NE = m->NE;
  m->nf = p.n_flavor;
  const double dE = (p.e_max_mev - p.e_min_mev) / (double)NE;
  const double du = 1.0 / (double)m->NU;
  m->h = (p.r_end_km - p.r_start_km) / (double)p.n_steps;
  const double s2gf = potential_per_density();
  m->lam0 = s2gf * p.n0_cm3;
  const double rcm = p.r_nu_km * 1.0e5;
  m->kappa0 = s2gf / (((2.0 * kPi) * (rcm * rcm)) * kClight);
  // [3]: anti-nu_x, with its own spectrum or that of nu_x
  double N[4], T[4];
  for (int a = 0; a < 3; ++a) T[a] = p.temp_mev[a];
  T[3] = (p.temp_xbar_mev != 0.0) ? p.temp_xbar_mev : p.temp_mev[2];
  const double Lxb = (p.temp_xbar_mev != 0.0) ? p.lum_xbar_erg_s : p.lum_erg_s[2];
  for (int a = 0; a < 3; ++a) N[a] = p.lum_erg_s[a] * kErgMeV / ((T[a] * kFD3) / kFD2);
  N[3] = Lxb * kErgMeV / ((T[3] * kFD3) / kFD2);
  // extended model: the azimuthal average (1/2pi) int dphi' becomes the mean over the bins
  const bool ext = p.n_phi > 0;
  const double pref = ext ? ((m->kappa0 * du) * dE) * (1.0 / (double)m->NP) : (m->kappa0 * du) * dE;
  const int nv = (m->nf == 2) ? 2 : kVacRows3;
  m->E.assign(NE, 0.0);
  // tables: [vacuum terms (2f: bx, bz; 3f: 6 entries and e_k = 1/E_k) | weights G_s of the
  // NS species rows] x NE, then (extended) cos and sin of the azimuth of every azimuthal bin
  const int NS = m->NS;
  m->tab.assign((size_t)(nv + NS) * NE + (ext ? (size_t)2 * m->NP : 0), 0.0);
  if (ext) {
    // bin midpoints phi_p = 2 pi (p + 1/2) / n_phi; for even n_phi the second half is the
    // first turned by pi with exactly flipped signs (azimuthal sums of an axially
    // symmetric state then vanish exactly)
    double* cp = m->tab.data() + (size_t)(nv + NS) * NE;
    double* sp = cp + m->NP;
    for (long long q = 0; q < m->NP; ++q) {
      if (m->NP % 2 == 0 && q >= m->NP / 2) {
        cp[q] = -cp[q - m->NP / 2];
        sp[q] = -sp[q - m->NP / 2];
      } else {
        const double ph = (2.0 * kPi) * (((double)q + 0.5) / (double)m->NP);
        cp[q] = std::cos(ph);
        sp[q] = std::sin(ph);
      }
    }
  }
  m->dtab.assign(m->nf == 2 ? (size_t)5 * NE : 0, 0.0);
  double* G0 = m->tab.data() + (size_t)nv * NE;
  double* G1 = G0 + NE;
  double U[3][3];
  if (m->nf == 3) {
    const double c12 = std::cos(p.theta[0]), s12 = std::sin(p.theta[0]);
    const double c13 = std::cos(p.theta[1]), s13 = std::sin(p.theta[1]);
    const double c23 = std::cos(p.theta[2]), s23 = std::sin(p.theta[2]);
    // U = R23 U13 R12 (delta = 0)
    U[0][0] = c12 * c13; U[0][1] = s12 * c13; U[0][2] = s13;
    U[1][0] = -(s12 * c23) - (c12 * s23) * s13; U[1][1] = c12 * c23 - (s12 * s23) * s13; U[1][2] = s23 * c13;
    U[2][0] = s12 * s23 - (c12 * c23) * s13; U[2][1] = -(c12 * s23) - (s12 * c23) * s13; U[2][2] = c23 * c13;
  }
  for (long long k = 0; k < NE; ++k) {
    const double e = p.e_min_mev + ((double)k + 0.5) * dE;
    m->E[k] = e;
    const double fe = fd_spectrum(e, p.temp_mev[0]);
    const double fb = fd_spectrum(e, p.temp_mev[1]);
    const double fx = fd_spectrum(e, p.temp_mev[2]);
    const double fxb = fd_spectrum(e, T[3]);
    if (NS == 2) {
      // heavy-flavour-born states are I - rho_e (unitarity): they enter with -N_x f_x
      // (antineutrinos: -N_xbar f_xbar)
      G0[k] = pref * (N[0] * fe - N[2] * fx);
      G1[k] = pref * (N[1] * fb - N[3] * fxb);
    } else {
      // every flavour tracked: species row s = anti * nf + flavour of birth
      for (int sp = 0; sp < NS; ++sp) {
        const int anti = sp / m->nf, fl = sp % m->nf;
        const double Nf = (fl == 0) ? (anti ? N[1] * fb : N[0] * fe) : (anti ? N[3] * fxb : N[2] * fx);
        G0[(size_t)sp * NE + k] = pref * Nf;
      }
    }
    if (m->nf == 2) {
      const double om = (kVac * p.dm2_ev2[0]) / e;
      const double s2 = std::sin(2.0 * p.theta[0]), c2 = std::cos(2.0 * p.theta[0]);
      m->tab[k] = (2.0 * om) * s2;            // B_vac,x
      m->tab[NE + k] = -((2.0 * om) * c2);    // B_vac,z
      // derivatives for the adjoint: dg/dL_a = pref f_a / <E_a> (erg -> MeV), the
      // heavy-flavour term entering both species with a minus sign; dB_vac/dtheta_v
      m->dtab[k] = pref * kErgMeV / ((p.temp_mev[0] * kFD3) / kFD2) * fe;
      m->dtab[NE + k] = pref * kErgMeV / ((p.temp_mev[1] * kFD3) / kFD2) * fb;
      m->dtab[2 * NE + k] = -(pref * kErgMeV / ((p.temp_mev[2] * kFD3) / kFD2) * fx);
      m->dtab[3 * NE + k] = (4.0 * om) * c2;
      m->dtab[4 * NE + k] = (4.0 * om) * s2;
    } else {
      const double w2 = ((2.0 * kVac) * p.dm2_ev2[0]) / e;  // dm^2_21 / 2E
      const double w3 = ((2.0 * kVac) * p.dm2_ev2[1]) / e;  // dm^2_31 / 2E
      static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
      for (int q = 0; q < 6; ++q) {
        m->tab[(size_t)q * NE + k] = (U[ia[q]][1] * U[ib[q]][1]) * w2 + (U[ia[q]][2] * U[ib[q]][2]) * w3;
        m->v0[q] = (U[ia[q]][1] * U[ib[q]][1]) * ((2.0 * kVac) * p.dm2_ev2[0]) +
                   (U[ia[q]][2] * U[ib[q]][2]) * ((2.0 * kVac) * p.dm2_ev2[1]);
      }
      m->tab[(size_t)6 * NE + k] = 1.0 / e;
    }
  }
  // largest sum of |entries| of the traceless vacuum Hamiltonian over the energy bins
  m->vac_max = 0.0;
  if (m->nf == 3) {
    for (long long k = 0; k < NE; ++k) {
      const double tr = (m->tab[k] + m->tab[NE + k] + m->tab[2 * NE + k]) / 3.0;
      double sv = 0.0;
      for (int q = 0; q < 3; ++q) sv += std::fabs(m->tab[(size_t)q * NE + k] - tr);
      for (int q = 3; q < 6; ++q) sv += 2.0 * std::fabs(m->tab[(size_t)q * NE + k]);
      m->vac_max = std::max(m->vac_max, sv);
    }
  }
  // fixed point: |g| 2^e1 < 2^50, so a beam contribution g rho~ 2^e1 of a state with
  // squared norm below 2 (checked per beam) stays below 2^51, where the fma with 1.5 2^52
  // rounds it exactly to an integer; a lane adds up to 32 of them in a 64-bit integer;
  // every angle term of J0, (energy sum / cos) 2^e0, stays below 2^62
  // (cos is smallest at r_start, u_max)
  double wmax = 0.0;
  for (long long i = 0; i < (long long)NS * NE; ++i) wmax = std::max(wmax, std::fabs(G0[i]));
  if (!(wmax > 0.0)) wmax = 1.0;
  int ex = 0;
  std::frexp(wmax, &ex);
  m->e1 = 50 - ex;
  const double qs = p.r_nu_km / p.r_start_km;
  const double ulast = ((double)(m->NU - 1) + 0.5) / (double)m->NU;
  const double cmin = std::sqrt(1.0 - ulast * (qs * qs));
  const double b0 = (wmax * (double)NE) * (1.0 / cmin);
  std::frexp(b0, &ex);
  m->e0 = 61 - ex;
  m->s1 = std::ldexp(1.0, m->e1);
  m->p2e1 = std::ldexp(1.0, -m->e1);
  m->s0 = std::ldexp(1.0, m->e0);
  m->p2e0 = std::ldexp(1.0, -m->e0);
  // Mixed precision (3f, FP32 state): the first step from which every beam's stage
  // generator rotates by at most one radian, bounded a priori by
  //   (h/c_min) (lambda + 8 mu G (1/c_min - c_min) + max_k sum |H_vac - tr/3|),
  // G = sum_b |g_b|: each nu-nu component mu |sum_b g_b rho~_b (1/c_b - c)| is at most
  // mu G (1/c_min - c_min) since |rho~| <= 1 and 0 <= 1/c_b - c <= 1/c_min - c_min.  Every
  // term decreases with r.
  m->fp32_from = p.n_steps;
  if (m->nf == 3) {
    double gsum = 0.0;
    for (long long i = 0; i < (long long)NS * NE; ++i) gsum += std::fabs(G0[i]);
    gsum *= (double)m->NU;
    long long last_bad = -1;
    for (long long n = 0; n < p.n_steps; ++n) {
      const double r = p.r_start_km + (double)n * m->h;
      const double q = p.r_nu_km / r;
      double qp = 1.0;
      for (int i = 0; i < p.ne_power; ++i) qp *= q;
      const double lam = m->lam0 * qp, mu = 0.5 * q * q;
      const double cmn = std::sqrt(1.0 - ulast * q * q);
      const double bound = (m->h / cmn) * ((lam + 8.0 * mu * gsum * (1.0 / cmn - cmn)) + m->vac_max);
      if (!(bound <= 1.0)) last_bad = n;
    }
    m->fp32_from = last_bad + 1;
  }
}

static int make_sub(const nb_params* p, Sub* s) {
  int rc = validate(p);
  if (rc) return rc;
  s->p = *p;
  s->NE = p->n_energy;
  s->NU = p->n_u;
  s->NP = (p->n_phi > 0) ? p->n_phi : 1;
  s->NS = p->track_all ? 2 * p->n_flavor : 2;
  build_tables(s);
  return NB_OK;
}

static nb_model* new_model(const nb_params* p) {
  nb_model* m = new (std::nothrow) nb_model();
  if (!m) return nullptr;
  m->p = *p;
  m->nf = p->n_flavor;
  m->nc = (m->nf == 2) ? 3 : 8;
  m->nsc = (m->nf == 2) ? 3 : 6;
  return m;
}

static void finish_layout_host(nb_model* m) {
  long long beam = 0, row = 0, t = 0;
  m->tab.clear();
  for (Sub& s : m->subs) {
    s.beam0 = beam;
    s.row0 = row;
    s.tab0 = t;
    beam += (long long)s.NS * s.NE * s.NU * s.NP;
    row += (long long)s.NS * s.NU * s.NP;
    t += (long long)s.tab.size();
    m->tab.insert(m->tab.end(), s.tab.begin(), s.tab.end());
  }
  m->nb = beam;
  m->rows = row;
  m->plane = (m->nb + 63) / 64 * 64;
  m->nmodels = (int)m->subs.size();
}

extern "C" int nb_model_create(const nb_params* p, nb_model** out) {
  if (!out) return fail(NB_EINVAL, "out is NULL");
  *out = nullptr;
  Sub s;
  int rc = make_sub(p, &s);
  if (rc) return rc;
  nb_model* m = new_model(p);
  if (!m) return fail(NB_EINVAL, "out of host memory");
  m->subs.push_back(std::move(s));
  finish_layout_host(m);
  *out = m;
  return NB_OK;
}

extern "C" int nb_batch_create(const nb_params* p, int32_t n_models, nb_model** out) {
  if (!out) return fail(NB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p || n_models < 1) return fail(NB_EINVAL, "need at least one model");
  std::vector<Sub> subs((size_t)n_models);
  for (int i = 0; i < n_models; ++i) {
    const nb_params& q = p[i];
    if (q.n_flavor != 2 || q.precision != NB_FP64)
      return fail(NB_EINVAL, "batched models are two-flavour FP64 (model %d)", i);
    if (q.adjoint_ckpt != 0) return fail(NB_EINVAL, "batched models have no adjoint (model %d)", i);
    if (q.adaptive != 0) return fail(NB_EINVAL, "batched models step on a fixed grid (model %d)", i);
    if (q.n_phi != 0) return fail(NB_EINVAL, "batched models are bulb models (model %d)", i);
    if (q.track_all != 0) return fail(NB_EINVAL, "batched models track two species (model %d)", i);
    if (q.n_steps != p[0].n_steps || q.r_start_km != p[0].r_start_km || q.r_end_km != p[0].r_end_km ||
        q.r_nu_km != p[0].r_nu_km || q.ne_power != p[0].ne_power || q.renorm != p[0].renorm)
      return fail(NB_EINVAL, "batched models must share the radial grid, R, ne_power and renorm (model %d)", i);
    int rc = make_sub(&q, &subs[i]);
    if (rc) return rc;
  }
  nb_model* m = new_model(p);
  if (!m) return fail(NB_EINVAL, "out of host memory");
  m->batch = true;
  m->subs = std::move(subs);
  finish_layout_host(m);
  *out = m;
  return NB_OK;
}

static void drop_graph(nb_model* m) {
  if (m->graph_exec) (void)hipGraphExecDestroy(m->graph_exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->graph_exec = nullptr;
  m->graph = nullptr;
  m->graph_steps = 0;
}

extern "C" void nb_model_destroy(nb_model* m) {
  if (!m) return;
  drop_graph(m);
  if (m->pinned) (void)hipHostFree(m->pinned);
  cancel_word_give(m->cancel);
  delete m;
}

extern "C" int64_t nb_n_beams(const nb_model* m) { return m ? m->nb : 0; }
extern "C" int32_t nb_n_models(const nb_model* m) { return m ? m->nmodels : 0; }
extern "C" int32_t nb_state_comps(const nb_model* m) { return m ? m->nsc : 0; }
extern "C" int64_t nb_step_index(const nb_model* m) { return m ? m->step : -1; }
extern "C" int64_t nb_mixed_fp32_step(const nb_model* m) {
  if (!m || m->batch || !state_fp32(m)) return -1;
  return m->subs[0].fp32_from;
}

extern "C" int nb_pee_offsets(const nb_model* m, int64_t* off) {
  if (!m || !off) return fail(NB_EINVAL, "NULL argument");
  for (int i = 0; i < m->nmodels; ++i) off[i] = m->subs[i].beam0;
  off[m->nmodels] = m->nb;
  return NB_OK;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace: state planes | tables | sync and tagged reduction words | step counter |
// (batches) model descriptors | wave row ranges | moment accumulators | (adjoint) its
// regions | (adaptive) the second state buffer.
struct Layout {
  size_t X, tab, sync, ctl, models, waves, acc, adj, spill, jhist, dtab, aout, X2, need;
};

// The adjoint (single two-flavour model with adjoint_ckpt = K > 0) reserves state slots
// for ceil(n_steps / K) checkpoints plus a tape of K states, the recorded stage moments of
// every step, its derivative tables, block partials and its outputs.
static bool adjoint_enabled(const nb_model* m) { return !m->batch && m->nf == 2 && m->p.adjoint_ckpt > 0; }
static long long adjoint_slots(const nb_model* m) {
  const long long K = m->p.adjoint_ckpt, N = m->p.n_steps;
  return (N + K - 1) / K + std::min(K, N);
}

static Layout layout_of(const nb_model* m) {
  const size_t es = state_fp32(m) ? sizeof(float) : sizeof(double);
  Layout L{};
  size_t o = 0;
  L.X = o;
  o = align256(o + es * (size_t)m->plane * m->nsc);
  L.tab = o;
  o = align256(o + sizeof(double) * m->tab.size());
  L.sync = o;
  o = align256(o + sizeof(unsigned int) * kSyncWords);
  L.ctl = o;
  o = align256(o + sizeof(long long) * kCtlWords);
  L.models = o;
  L.waves = o;
  L.acc = o;
  if (m->batch) {
    o = align256(o + sizeof(BatchModel) * (size_t)m->nmodels);
    L.waves = o;
    o = align256(o + sizeof(long long) * ((size_t)kMaxBlocks * (kBlock / 64) + 1));
    L.acc = o;
    o = align256(o + sizeof(unsigned long long) * (size_t)kAccSets * m->nmodels * 6 * kAccLimbs);
  }
  L.adj = L.jhist = L.dtab = L.aout = L.spill = o;
  if (adjoint_enabled(m)) {
    o = align256(o + sizeof(double) * (size_t)adjoint_slots(m) * 3 * m->plane);
    L.spill = o;   // the reverse kernel's adjoint registers when the beams outnumber its threads
    o = align256(o + sizeof(double) * (size_t)9 * m->plane);
    L.jhist = o;
    o = align256(o + sizeof(double) * (size_t)(m->p.n_steps + 1) * 24);
    L.dtab = o;
    o = align256(o + sizeof(double) * m->subs[0].dtab.size());
    L.aout = o;
    o = align256(o + sizeof(double) * 8);
  }
  L.X2 = o;
  if (!m->batch && m->p.adaptive) o = align256(o + es * (size_t)m->plane * m->nsc);
  L.need = o;
  return L;
}

extern "C" size_t nb_workspace_bytes(const nb_model* m) { return m ? layout_of(m).need : 0; }

// Energy tables are staged in LDS when they fit in this many bytes per block (the
// stepping kernels' static LDS is about 50 KB; a CU holds 160 KB and runs one block).
static constexpr size_t kTabLdsMax = 96 * 1024;

static size_t tab_bytes(const nb_model* m) { return sizeof(double) * m->tab.size(); }
static bool tab_in_lds(const nb_model* m) { return !m->batch && tab_bytes(m) <= kTabLdsMax; }
static size_t advance_dyn_lds(const nb_model* m) { return tab_in_lds(m) ? tab_bytes(m) : 0; }
// The FP32-arithmetic kernel stages the table and, from the next 16-byte boundary, an FP32
// copy of the vacuum rows and e_k (eight floats per energy) when both fit in this many
// bytes (with its static LDS, below the 160 KB of a CU).
static constexpr size_t kTabLdsMaxF32 = 104 * 1024;
static size_t f32_lds_bytes(const nb_model* m) {
  return sizeof(double) * ((m->tab.size() + 1) & ~(size_t)1) + sizeof(float) * 8 * (size_t)m->p.n_energy;
}
static bool f32_tab_in_lds(const nb_model* m) { return !m->batch && f32_lds_bytes(m) <= kTabLdsMaxF32; }
static size_t f32_dyn_lds(const nb_model* m) { return f32_tab_in_lds(m) ? f32_lds_bytes(m) : 0; }

// The adaptive-step kernel of a single FP64 model created with adaptive = 1 (else nullptr).
static const void* adaptive_kernel(const nb_model* m) {
  if (m->batch || !m->p.adaptive) return nullptr;
  const bool l = tab_in_lds(m);
  if (m->nf == 2) return l ? (const void*)&k_adaptive<2, true> : (const void*)&k_adaptive<2, false>;
  return l ? (const void*)&k_adaptive<3, true> : (const void*)&k_adaptive<3, false>;
}

// Packed row tails (k_advance<..., PK = true>): three flavours with FP64 state and
// arithmetic, the bulb model, 512 threads, one row per wavefront of a launch of nblocks
// blocks, N_E = 64 m + t with 1 <= t <= 32 and N_E <= 2048.  The kernel ends with a range
// error (it does not wait) if launched otherwise.
static bool packed_tails(const nb_model* m, int nblocks) {
  const long long ne = m->p.n_energy;
  return !m->batch && m->nf == 3 && !state_fp32(m) && m->p.n_phi == 0 && nblocks > 0 &&
         (long long)nblocks * (kBlock / 64) == m->rows && ne > 64 && ne <= 64 * 32 && (ne % 64) != 0 &&
         (ne % 64) <= 32;
}
static const void* packed_kernel(const nb_model* m) {
  return tab_in_lds(m) ? (const void*)&k_advance<3, double, true, false, false, kBlock, true>
                       : (const void*)&k_advance<3, double, false, false, false, kBlock, true>;
}
// The fixed-step kernel of a model at bs threads per block (512 or 256).
template <int BS>
static const void* advance_kernel_bs(const nb_model* m) {
  if (m->batch) return (const void*)&k_batch2<BS>;
  const bool l = tab_in_lds(m);
  if (m->nf == 2)
    return m->p.n_phi > 0
               ? (l ? (const void*)&k_advance<2, double, true, false, true, BS, false> : (const void*)&k_advance<2, double, false, false, true, BS, false>)
               : (l ? (const void*)&k_advance<2, double, true, false, false, BS, false> : (const void*)&k_advance<2, double, false, false, false, BS, false>);
  if (state_fp32(m))
    return l ? (const void*)&k_advance<3, float, true, false, false, BS, false> : (const void*)&k_advance<3, float, false, false, false, BS, false>;
  if (m->p.n_phi > 0)
    return l ? (const void*)&k_advance<3, double, true, false, true, BS, false> : (const void*)&k_advance<3, double, false, false, true, BS, false>;
  if constexpr (BS == kBlock) {
    if (packed_tails(m, m->nblocks)) return packed_kernel(m);
  }
  return l ? (const void*)&k_advance<3, double, true, false, false, BS, false> : (const void*)&k_advance<3, double, false, false, false, BS, false>;
}
static const void* advance_kernel(const nb_model* m, int bs) {
  return bs == kBlockSmall ? advance_kernel_bs<kBlockSmall>(m) : advance_kernel_bs<kBlock>(m);
}
// The FP32-arithmetic stepping kernel of the mixed-precision mode (nullptr otherwise).
static const void* advance_kernel_f32(const nb_model* m, int bs) {
  if (m->batch || !state_fp32(m)) return nullptr;
  if (bs == kBlockSmall)
    return f32_tab_in_lds(m) ? (const void*)&k_advance<3, float, true, true, false, kBlockSmall, false>
                             : (const void*)&k_advance<3, float, false, true, false, kBlockSmall, false>;
  return f32_tab_in_lds(m) ? (const void*)&k_advance<3, float, true, true, false, kBlock, false>
                           : (const void*)&k_advance<3, float, false, true, false, kBlock, false>;
}

static int launch_1d(const void* fn, long long n, void** args, hipStream_t s) {
  const int bs = 256;
  const long long nblk = (n + bs - 1) / bs;
  if (nblk <= 0) return NB_OK;
  NB_HIP(hipLaunchKernel(fn, dim3((unsigned)nblk), dim3(bs), args, 0, s));
  return NB_OK;
}

static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

static int set_device_step(nb_model* m, long long step) {
  long long* ctl = (long long*)(m->ws + m->off_ctl);
  void* args[] = {&ctl, &step};
  NB_HIP(hipLaunchKernel((const void*)&k_set_step, dim3(1), dim3(1), args, 0, m->stream));
  return NB_OK;
}

// Clear the barrier words, optionally keeping the status word (a kernel: capturable).
static int zero_sync(nb_model* m, int keep) {
  unsigned int* sync = sync_words(m);
  const unsigned* cancel = m->cancel_dev;
  void* zargs[] = {&sync, &keep, &cancel};
  NB_HIP(hipLaunchKernel((const void*)&k_zero_sync, dim3(256), dim3(256), zargs, 0, m->stream));
  return NB_OK;
}

extern "C" int nb_reset(nb_model* m) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  void* X = m->ws + m->off_X;
  long long nb_ = m->nb, plane = m->plane;
  int nsc = m->nsc;
  // flavour of birth: species row s of a single model = anti * (NS/2) + flavour; batches and
  // two tracked species are all electron-born
  const Sub& s0 = m->subs[0];
  long long per_species = m->batch ? m->nb : s0.NE * s0.NU * s0.NP;
  int nfl = m->batch ? 1 : s0.NS / 2;
  void* args[] = {&X, &nb_, &plane, &nsc, &per_species, &nfl};
  int rc = launch_1d(state_fp32(m) ? (const void*)&k_init<float> : (const void*)&k_init<double>,
                     m->nb, args, m->stream);
  if (rc) return rc;
  rc = set_device_step(m, 0);
  if (rc) return rc;
  m->step = 0;
  return NB_OK;
}

// Resident blocks of the fixed-step kernels at bs threads per block (bind-time occupancy).
static int capacity(const nb_model* m, int bs) { return bs == kBlockSmall ? m->cap256 : m->cap512; }
// Blocks of one fixed-step launch at bs threads per block: at most one wavefront per row, at
// most the resident capacity, at most cap (> 0).
static int blocks_for(const nb_model* m, int bs, int cap) {
  const int wpb = bs / 64;
  const long long want = (m->rows + wpb - 1) / wpb;
  int nb_ = (int)std::min<long long>(want, capacity(m, bs));
  if (cap > 0) nb_ = std::min(nb_, cap);
  return std::max(1, nb_);
}
static int launch_blocks(const nb_model* m) { return blocks_for(m, m->bs, m->tune_blocks); }

// Contiguous row ranges per wavefront with balanced cost (64-lane chunks + row overhead).
static int upload_partition(nb_model* m) {
  const int waves = m->nblocks * (m->bs / 64);
  std::vector<double> cost;
  double total = 0.0;
  for (const Sub& s : m->subs) {
    const double c = (double)((s.NE + 63) / 64) + m->tune_row_cost;
    total += c * 2.0 * (double)s.NU;
  }
  std::vector<long long> w0((size_t)waves + 1, m->rows);
  long long row = 0;
  double acc = 0.0;
  int w = 0;
  w0[0] = 0;
  for (const Sub& s : m->subs) {
    const double c = (double)((s.NE + 63) / 64) + m->tune_row_cost;
    for (long long r = 0; r < 2LL * s.NU; ++r, ++row) {
      while (w + 1 <= waves && acc >= total * (double)(w + 1) / (double)waves) w0[(size_t)(++w)] = row;
      acc += c;
    }
  }
  for (int i = w + 1; i <= waves; ++i) w0[(size_t)i] = m->rows;
  NB_HIP(hipMemcpyAsync(m->ws + m->off_waves, w0.data(), sizeof(long long) * w0.size(),
                        hipMemcpyHostToDevice, m->stream));
  NB_HIP(hipStreamSynchronize(m->stream));
  return NB_OK;
}

// Resident blocks of the model's fixed-step kernels at bs threads per block: the least
// per-CU occupancy over the kernels its launches use (with their dynamic LDS) times the CUs,
// at most kMaxBlocks and p.max_blocks; 0 if one of them cannot be resident at that size.
static int fixed_step_capacity(const nb_model* m, int cus, int bs, int* out) {
  int per = 0;
  NB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, advance_kernel(m, bs), bs, advance_dyn_lds(m)));
  if (bs == kBlock && !m->batch && m->nf == 3 && !state_fp32(m) && m->p.n_phi == 0) {
    int ppk = 0;   // the packed-tail variant may take any of these launches
    NB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&ppk, packed_kernel(m), bs, advance_dyn_lds(m)));
    per = std::min(per, ppk);
  }
  if (advance_kernel_f32(m, bs)) {
    int p32 = 0;
    NB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&p32, advance_kernel_f32(m, bs), bs, f32_dyn_lds(m)));
    per = std::min(per, p32);
  }
  int cap = std::min(cus * per, kMaxBlocks);
  if (m->p.max_blocks > 0) cap = std::min(cap, (int)m->p.max_blocks);
  *out = std::max(0, cap);
  return NB_OK;
}

extern "C" int nb_bind(nb_model* m, void* dev_ws, size_t bytes, void* hip_stream) {
  if (!m || !dev_ws) return fail(NB_EINVAL, "NULL model or workspace");
  if (((uintptr_t)dev_ws) % 256) return fail(NB_EWORKSPACE, "workspace must be 256-byte aligned");
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  int cus = 0, khz = 0;
  NB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  NB_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  int cap[2] = {0, 0}, cap_adaptive = 0;
  for (int i = 0; i < 2; ++i) {
    int rc = fixed_step_capacity(m, cus, i == 0 ? kBlock : kBlockSmall, &cap[i]);
    if (rc) return rc;
  }
  if (cap[0] < 1) return fail(NB_EHIP, "stepping kernel cannot be resident");
  if (adaptive_kernel(m)) {
    int nba = 0;
    NB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nba, adaptive_kernel(m), kBlock,
                                                         advance_dyn_lds(m)));
    if (nba < 1) return fail(NB_EHIP, "adaptive kernel cannot be resident");
    cap_adaptive = std::min(cus * nba, kMaxBlocks);
    if (m->p.max_blocks > 0) cap_adaptive = std::min(cap_adaptive, (int)m->p.max_blocks);
  }
  const Layout L = layout_of(m);
  if (bytes < L.need)
    return fail(NB_EWORKSPACE, "workspace too small: %zu < %zu bytes", bytes, L.need);
  drop_graph(m);
  m->off_X = L.X;
  m->off_tab = L.tab;
  m->off_sync = L.sync;
  m->off_ctl = L.ctl;
  m->off_models = L.models;
  m->off_waves = L.waves;
  m->off_acc = L.acc;
  m->off_adj = L.adj;
  m->off_spill = L.spill;
  m->off_jhist = L.jhist;
  m->off_dtab = L.dtab;
  m->off_aout = L.aout;
  m->off_X2 = L.X2;
  m->need = L.need;
  m->adj_bpt = 0;
  m->adj_blocks = 0;
  if (adjoint_enabled(m)) {
    // smallest beams-per-thread variant whose resident grid covers every beam; beyond four
    // beams per resident thread, the spill variant (adjoint registers in the workspace) on
    // the full resident grid
    static const int bpts[3] = {1, 2, 4};
    static const void* fns[3] = {(const void*)&k_adjoint2<1>, (const void*)&k_adjoint2<2>,
                                 (const void*)&k_adjoint2<4>};
    for (int i = 0; i < 3 && !m->adj_bpt; ++i) {
      int per = 0;
      NB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fns[i], kBlock, 0));
      int blocks = std::min(cus * per, kMaxBlocks);
      if (m->p.max_blocks > 0) blocks = std::min(blocks, (int)m->p.max_blocks);
      const long long need_blocks = (m->nb + (long long)bpts[i] * kBlock - 1) / ((long long)bpts[i] * kBlock);
      if (per >= 1 && need_blocks <= blocks) {
        m->adj_bpt = bpts[i];
        m->adj_blocks = (int)std::max<long long>(1, need_blocks);
      }
    }
    if (!m->adj_bpt) {
      int per = 0;
      NB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)&k_adjoint2<0>, kBlock, 0));
      if (per < 1) return fail(NB_EHIP, "adjoint kernel cannot be resident");
      int blocks = std::min(cus * per, kMaxBlocks);
      if (m->p.max_blocks > 0) blocks = std::min(blocks, (int)m->p.max_blocks);
      m->adj_bpt = -1;   // spill mode
      m->adj_blocks = std::max(1, blocks);
    }
  }
  m->ws = (char*)dev_ws;
  m->ws_bytes = bytes;
  m->stream = (hipStream_t)hip_stream;
  m->device = dev;
  m->cus = cus;
  m->cap512 = cap[0];
  m->cap256 = cap[1];
  m->cap_adaptive = cap_adaptive;
  // Default shape: two flavours (single, batched or extended) at 256 threads per block
  // (three wavefronts per SIMD, and small models spread over twice as many CUs: 16 % faster
  // on the 256-model batch and the 200k model, 9 % on the 60M extended model); three
  // flavours at 512 (the 256-thread variant measured 19 % slower on the 800k model).
  if (!m->tuned) m->bs = (m->nf == 2 && m->cap256 > 0) ? kBlockSmall : kBlock;
  if (capacity(m, m->bs) < 1) m->bs = kBlock;   // a tuned block size this device cannot hold
  if (m->tune_blocks > capacity(m, m->bs)) m->tune_blocks = 0;
  m->nblocks = launch_blocks(m);
  if (!m->cancel) {
    int rc = cancel_word_take(&m->cancel, &m->cancel_dev);
    if (rc) return rc;
  }
  m->ticks_per_s = (unsigned long long)(khz > 0 ? khz : 100000) * 1000ull;
  if (!m->pinned) NB_HIP(hipHostMalloc((void**)&m->pinned, 256, hipHostMallocDefault));
  NB_HIP(hipMemcpyAsync(m->ws + m->off_tab, m->tab.data(), tab_bytes(m), hipMemcpyHostToDevice,
                        m->stream));
  if (adjoint_enabled(m))
    NB_HIP(hipMemcpyAsync(m->ws + m->off_dtab, m->subs[0].dtab.data(), sizeof(double) * m->subs[0].dtab.size(),
                          hipMemcpyHostToDevice, m->stream));
  if (m->batch) {
    std::vector<BatchModel> md((size_t)m->nmodels);
    for (int i = 0; i < m->nmodels; ++i) {
      const Sub& s = m->subs[i];
      md[i] = BatchModel{s.beam0, s.row0, s.tab0, (int)s.NE, (int)s.NU, s.lam0, s.s1, s.s0, s.p2e1, s.p2e0};
    }
    NB_HIP(hipMemcpyAsync(m->ws + m->off_models, md.data(), sizeof(BatchModel) * md.size(),
                          hipMemcpyHostToDevice, m->stream));
    NB_HIP(hipStreamSynchronize(m->stream));
    int rc = upload_partition(m);
    if (rc) return rc;
  }
  unsigned int* sync = (unsigned int*)(m->ws + m->off_sync);
  int keep = 0;
  const unsigned* no_cancel = nullptr;
  void* zargs[] = {&sync, &keep, &no_cancel};
  NB_HIP(hipLaunchKernel((const void*)&k_zero_sync, dim3(256), dim3(256), zargs, 0, m->stream));
  NB_HIP(hipStreamSynchronize(m->stream));
  return nb_reset(m);
}

// Read and clear the kernels' status word and read back the device step counter (only
// outside graph capture).
static int check_status(nb_model* m) {
  if (capturing(m->stream)) return NB_OK;
  unsigned int* sync = sync_words(m);
  const long long* ctl = (const long long*)(m->ws + m->off_ctl);
  long long* host = m->pinned;
  void* sargs[] = {&sync, &ctl, &host};
  NB_HIP(hipLaunchKernel((const void*)&k_status_out, dim3(1), dim3(1), sargs, 0, m->stream));
  NB_HIP(hipStreamSynchronize(m->stream));
  const unsigned st = (unsigned)(m->pinned[0] & 0xffffffffll);
  m->step = m->pinned[1];
  if (st) {
    int keep = 0;
    const unsigned* no_cancel = nullptr;
    void* zargs[] = {&sync, &keep, &no_cancel};
    NB_HIP(hipLaunchKernel((const void*)&k_zero_sync, dim3(256), dim3(256), zargs, 0, m->stream));
    NB_HIP(hipStreamSynchronize(m->stream));
    if (st & 4u) return fail(NB_ETIMEOUT, "cancelled by the host (nb_cancel)");
    if (st & 2u) return fail(NB_ETIMEOUT, "grid barrier time limit exceeded");
    if (st & 8u)
      return fail(NB_ENUMERIC, "renormalisation factor far from 1 (|state|^2 off 1 by more than %g)",
                  state_fp32(m) ? 1e-5 : 1e-8);
    return fail(NB_ENUMERIC, "moment contribution out of fixed-point range (NaN or overflow)");
  }
  return NB_OK;
}

// Largest step count of one launch: keeps the barrier epochs inside 32 bits.
static long long launch_chunk(const nb_model* m) {
  return std::max<long long>(1, (long long)(3.5e9 / ((double)m->nblocks * 4.0)) - 2);
}

// Persistent launches (stepping, adaptive, adjoint) are ordinary launches whose grid never
// exceeds the resident capacity measured at nb_bind (one block per CU slot the occupancy
// calculator reports; a graph launch checks it again), so every block is resident while no
// other work holds the CUs, and every barrier wait is time-limited and cancellable from the
// host.  hipLaunchCooperativeKernel would only repeat the capacity check: on this runtime it
// cost 15-18 us more per call, and processes that had made cooperative launches crashed in
// the runtime's exit handler under rocprofv3 (ordinary launches exit cleanly).
//
// Enqueue one stepping launch of k steps (from the device step counter) on the stream.
static int enqueue_advance(nb_model* m, long long k) {
  unsigned int* sync = sync_words(m);
  int rc0 = zero_sync(m, 1);
  if (rc0) return rc0;
  const unsigned long long timeout = m->ticks_per_s * 20ull;
  if (m->batch) {
    unsigned long long* acc = acc_words(m);
    long long nacc = (long long)kAccSets * m->nmodels * 6 * kAccLimbs;
    void* zz[] = {&acc, &nacc};
    NB_HIP(hipLaunchKernel((const void*)&k_zero_u64, dim3(64), dim3(256), zz, 0, m->stream));
    BatchArgs a{};
    a.X = (double*)(m->ws + m->off_X);
    a.plane = m->plane;
    a.tab = (const double*)(m->ws + m->off_tab);
    a.models = (const BatchModel*)(m->ws + m->off_models);
    a.nmodels = m->nmodels;
    a.wave_row0 = (const long long*)(m->ws + m->off_waves);
    a.total_rows = m->rows;
    a.acc = acc;
    a.sync = sync;
    a.step_ctl = (long long*)(m->ws + m->off_ctl);
    a.nsteps = k;
    a.total_steps = m->p.n_steps;
    a.rs = m->p.r_start_km;
    a.h = m->subs[0].h;
    a.R = m->p.r_nu_km;
    a.ne_power = m->p.ne_power;
    a.renorm = m->p.renorm;
    a.timeout_ticks = timeout;
    a.cancel = m->cancel_dev;
    void* args[] = {&a};
    const hipError_t e =
        hipLaunchKernel(advance_kernel(m, m->bs), dim3(m->nblocks), dim3(m->bs), args, 0, m->stream);
    if (e != hipSuccess) return fail(NB_EHIP, "batch launch: %s", hipGetErrorString(e));
    return NB_OK;
  }
  const Sub& s = m->subs[0];
  StepArgs a{};
  a.X = m->ws + m->off_X;
  a.tab = (const double*)(m->ws + m->off_tab);
  a.sync = sync;
  a.step_ctl = (long long*)(m->ws + m->off_ctl);
  a.plane = m->plane;
  a.NE = (int)s.NE;
  a.NU = (int)s.NU;
  a.NP = (int)s.NP;
  a.NS = s.NS;
  a.nsteps = k;
  a.total_steps = m->p.n_steps;
  a.rs = m->p.r_start_km;
  a.h = s.h;
  a.R = m->p.r_nu_km;
  a.lam0 = s.lam0;
  a.ne_power = m->p.ne_power;
  a.renorm = m->p.renorm;
  a.s1 = s.s1;
  a.s0 = s.s0;
  a.p2e1 = s.p2e1;
  a.p2e0 = s.p2e0;
  for (int q = 0; q < 6; ++q) a.v0[q] = s.v0[q];
  a.timeout_ticks = timeout;
  a.cancel = m->cancel_dev;
  a.Jhist = m->jhist;
  auto launch = [&](const void* fn, size_t lds) -> int {
    void* args[] = {&a};
    const hipError_t e = hipLaunchKernel(fn, dim3(m->nblocks), dim3(m->bs), args, lds, m->stream);
    if (e != hipSuccess) return fail(NB_EHIP, "stepping launch: %s", hipGetErrorString(e));
    return NB_OK;
  };
  if (!advance_kernel_f32(m, m->bs)) return launch(advance_kernel(m, m->bs), advance_dyn_lds(m));
  // Mixed precision: FP64-arithmetic steps before fp32_from, FP32-arithmetic steps after,
  // as two windowed launches sharing one target of k steps from the device counter.
  {
    long long* ctl = (long long*)(m->ws + m->off_ctl);
    long long kk = k, total = m->p.n_steps;
    void* targs[] = {&ctl, &kk, &total};
    NB_HIP(hipLaunchKernel((const void*)&k_set_target, dim3(1), dim3(1), targs, 0, m->stream));
  }
  a.use_window = 1;
  a.win_lo = 0;
  a.win_hi = s.fp32_from;
  int rc = launch(advance_kernel(m, m->bs), advance_dyn_lds(m));
  if (rc) return rc;
  rc = zero_sync(m, 1);
  if (rc) return rc;
  a.win_lo = s.fp32_from;
  a.win_hi = m->p.n_steps;
  return launch(advance_kernel_f32(m, m->bs), f32_dyn_lds(m));
}

static int advance(nb_model* m, long long n) {
  const long long chunk = launch_chunk(m);
  while (n > 0) {
    const long long k = std::min(n, chunk);
    int rc = enqueue_advance(m, k);
    if (rc) return rc;
    n -= k;
    if (capturing(m->stream)) continue;
    const long long before = m->step;
    rc = check_status(m);
    if (rc) return rc;
    if (m->step != before + k) return fail(NB_EHIP, "device step counter out of step");
  }
  return NB_OK;
}

extern "C" int nb_step(nb_model* m, int64_t n) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (n < 0) return fail(NB_EINVAL, "negative step count");
  n = std::min<int64_t>(n, m->p.n_steps - m->step);
  if (n <= 0) return NB_OK;
  return advance(m, n);
}

extern "C" int nb_run(nb_model* m) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  return nb_step(m, m->p.n_steps - m->step);
}

// ------------------------------------------------- static scratch: stepping without allocation
// nb_step_static takes the scratch of the stepping launches -- the barrier and tagged
// reduction words (kSyncWords 32-bit words, enough for the largest grid of kMaxBlocks
// blocks) and the batch kernel's moment accumulators (kStaticModels models) -- from this
// array instead of the workspace.  Each device holds its own copy until the process ends.
constexpr int kStaticModels = 1024;
constexpr size_t kStaticSync64 = ((size_t)kSyncWords + 1) / 2;         // sync words, as u64
constexpr size_t kStaticAccOff = (kStaticSync64 + 31) / 32 * 32;       // 256-byte boundary
constexpr size_t kStaticWords = kStaticAccOff + (size_t)kAccSets * kStaticModels * 6 * kAccLimbs;
static __device__ __align__(256) unsigned long long scratch[kStaticWords];

// Device address of this device's copy of scratch, looked up once per device with that
// device current (the host-side name of the array is not a device address).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};
static int static_scratch(int dev, unsigned long long** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return fail(NB_EINVAL, "device %d out of range", dev);
  if (!g_scratch_addr[dev]) {
    int cur = 0;
    NB_HIP(hipGetDevice(&cur));
    if (cur != dev) NB_HIP(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
      return fail(NB_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_addr[dev] = ptr;
  }
  *out = (unsigned long long*)g_scratch_addr[dev];
  return NB_OK;
}

extern "C" int nb_step_static(nb_model* m, int64_t n) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (n < 0) return fail(NB_EINVAL, "negative step count");
  if (m->batch && m->nmodels > kStaticModels)
    return fail(NB_EINVAL, "nb_step_static: %d models exceed the static scratch limit of %d models",
                m->nmodels, kStaticModels);
  if (m->nblocks > kMaxBlocks)
    return fail(NB_EINVAL, "nb_step_static: %d blocks exceed the static scratch limit of %d blocks",
                m->nblocks, kMaxBlocks);
  unsigned long long* s = nullptr;
  int rc = static_scratch(m->device, &s);
  if (rc) return rc;
  m->sync_static = (unsigned int*)s;
  m->acc_static = s + kStaticAccOff;
  // the previous call on this device left its epochs (and maybe a status) in the array
  rc = zero_sync(m, 0);
  if (!rc) rc = nb_step(m, n);
  m->sync_static = nullptr;
  m->acc_static = nullptr;
  return rc;
}

// ----------------------------------------------------------------- adaptive steps
extern "C" int nb_run_adaptive(nb_model* m, double tol, double h_max_km, int64_t max_attempts,
                               nb_adaptive_stats* stats) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (!adaptive_kernel(m)) return fail(NB_EINVAL, "model was not created with adaptive = 1");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(NB_EINVAL, "tol must be > 0");
  if (max_attempts < 1) return fail(NB_EINVAL, "max_attempts must be >= 1");
  if (!std::isfinite(h_max_km)) return fail(NB_EINVAL, "h_max_km must be finite");
  if (m->step != 0) return fail(NB_EINVAL, "adaptive runs start at step 0 (call nb_reset)");
  if (capturing(m->stream)) return fail(NB_EINVAL, "adaptive runs cannot be captured");
  drop_graph(m);
  const Sub& s = m->subs[0];
  const double span = m->p.r_end_km - m->p.r_start_km;
  long long init[kCtlMKind + 1] = {};
  init[kCtlMTag] = -1;
  double r0 = m->p.r_start_km, h0 = s.h;
  std::memcpy(&init[kCtlR], &r0, sizeof(double));
  std::memcpy(&init[kCtlH], &h0, sizeof(double));
  long long* ctl = (long long*)(m->ws + m->off_ctl);
  NB_HIP(hipMemcpyAsync(ctl, init, sizeof(init), hipMemcpyHostToDevice, m->stream));
  int rc = zero_sync(m, 1);
  if (rc) return rc;
  StepArgs a{};
  a.X = m->ws + m->off_X;
  a.X2 = m->ws + m->off_X2;
  a.tab = (const double*)(m->ws + m->off_tab);
  a.sync = (unsigned int*)(m->ws + m->off_sync);
  a.step_ctl = ctl;
  a.plane = m->plane;
  a.NE = (int)s.NE;
  a.NU = (int)s.NU;
  a.NP = 1;
  a.NS = s.NS;
  a.nsteps = m->p.n_steps;
  a.total_steps = m->p.n_steps;
  a.rs = m->p.r_start_km;
  a.h = s.h;
  a.R = m->p.r_nu_km;
  a.lam0 = s.lam0;
  a.ne_power = m->p.ne_power;
  a.renorm = m->p.renorm;
  a.s1 = s.s1;
  a.s0 = s.s0;
  a.p2e1 = s.p2e1;
  a.p2e0 = s.p2e0;
  for (int q = 0; q < 6; ++q) a.v0[q] = s.v0[q];
  a.timeout_ticks = m->ticks_per_s * 20ull;
  a.cancel = m->cancel_dev;
  a.tol2 = tol * tol;
  a.hmax = (h_max_km > 0.0) ? h_max_km : span;
  a.hmin = std::ldexp(s.h, -40);
  a.r_end = m->p.r_end_km;
  a.max_attempts = max_attempts;
  void* args[] = {&a};
  // one wavefront per row at most, at most the adaptive kernel's resident capacity
  const int ablocks = (int)std::max<long long>(1, std::min<long long>((m->rows + 7) / 8, m->cap_adaptive));
  const hipError_t e = hipLaunchKernel(adaptive_kernel(m), dim3(ablocks), dim3(kBlock), args,
                                      advance_dyn_lds(m), m->stream);
  if (e != hipSuccess) return fail(NB_EHIP, "adaptive launch: %s", hipGetErrorString(e));
  long long out[8];
  NB_HIP(hipMemcpyAsync(out, ctl, sizeof(out), hipMemcpyDeviceToHost, m->stream));
  rc = check_status(m);
  if (rc) return rc;
  if (stats) {
    stats->accepted = out[kCtlAcc];
    stats->rejected = out[kCtlRej];
    stats->attempts = out[kCtlAtt];
    std::memcpy(&stats->h_last_km, &out[kCtlH], sizeof(double));
  }
  if (out[kCtlFail]) {
    // the partial state has no place on the fixed grid: back to the initial state
    rc = nb_reset(m);
    if (rc) return rc;
    return fail(NB_ESTEP, "adaptive step control failed after %lld attempts (%lld accepted)",
                (long long)out[kCtlAtt], (long long)out[kCtlAcc]);
  }
  return NB_OK;
}

// ----------------------------------------------------------------- HIP graphs
extern "C" int nb_graph_capture(nb_model* m, int64_t n_steps) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (n_steps < 1 || n_steps > launch_chunk(m)) return fail(NB_EINVAL, "bad step count for a graph");
  if (!m->stream) return fail(NB_EINVAL, "graph capture needs a non-default stream");
  drop_graph(m);
  NB_HIP(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_advance(m, n_steps);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(m->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(NB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&m->graph_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(NB_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  m->graph = g;
  m->graph_steps = n_steps;
  m->graph_bs = m->bs;
  m->graph_blocks = m->nblocks;
  return NB_OK;
}

extern "C" int nb_graph_launch(nb_model* m) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->graph_exec) return fail(NB_EINVAL, "no graph captured");
  // Inside the graph the persistent kernel is an ordinary launch, which makes progress only
  // if all its blocks are resident at once: check the recorded grid against the occupancy
  // the device reports now.
  int cur = 0, cus = 0, cap = 0;
  NB_HIP(hipGetDevice(&cur));
  if (cur != m->device) return fail(NB_EINVAL, "graph launch on device %d, model bound on %d", cur, m->device);
  NB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cur));
  int rc = fixed_step_capacity(m, cus, m->graph_bs, &cap);
  if (rc) return rc;
  if (m->graph_blocks > cap)
    return fail(NB_EINVAL, "captured grid of %d blocks of %d threads exceeds the resident capacity %d",
                m->graph_blocks, m->graph_bs, cap);
  NB_HIP(hipGraphLaunch(m->graph_exec, m->stream));
  return check_status(m);
}

extern "C" int nb_cancel(nb_model* m, int32_t on) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->cancel) return fail(NB_EUNBOUND, "no workspace bound");
  __atomic_store_n(m->cancel, on ? 1u : 0u, __ATOMIC_SEQ_CST);
  return NB_OK;
}

// ------------------------------------------------------------------ autotuner
// Launch shapes of the fixed-step kernels: threads per block (512 or 256), a block cap and,
// for batches, the per-row overhead of the cost model that splits the rows among
// wavefronts.  A beam's arithmetic does not depend on the shape and the moments are exact
// integer sums, so every shape gives the same bits.

// Shape -> model (bound, not capturing): block count and, for batches, the row partition.
static int apply_shape(nb_model* m, int bs, int blocks, double row_cost) {
  drop_graph(m);
  m->bs = bs;
  m->tuned = true;
  m->tune_blocks = blocks;
  m->tune_row_cost = row_cost;
  m->nblocks = launch_blocks(m);
  return m->batch ? upload_partition(m) : NB_OK;
}

static int check_shape(const nb_model* m, int bs, int blocks, double row_cost) {
  if (bs != kBlock && bs != kBlockSmall) return fail(NB_EINVAL, "block_threads must be 512 or 256");
  if (capacity(m, bs) < 1) return fail(NB_EINVAL, "the stepping kernels cannot be resident at %d threads", bs);
  if (blocks < 0 || blocks > capacity(m, bs))
    return fail(NB_EINVAL, "blocks must be in 0..%d (the resident capacity at %d threads)", capacity(m, bs), bs);
  if (m->batch && !(row_cost > 0.0 && row_cost < 1e6)) return fail(NB_EINVAL, "row_cost must be in (0, 1e6)");
  return NB_OK;
}

extern "C" int nb_set_tuning(nb_model* m, const nb_tuning* t) {
  if (!m || !t) return fail(NB_EINVAL, "NULL argument");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (capturing(m->stream)) return fail(NB_EINVAL, "the launch shape cannot change during capture");
  const double rc_ = m->batch ? t->row_cost : m->tune_row_cost;
  int rc = check_shape(m, t->block_threads, t->blocks, rc_);
  if (rc) return rc;
  return apply_shape(m, t->block_threads, t->blocks, rc_);
}

extern "C" int nb_get_tuning(const nb_model* m, nb_tuning* t) {
  if (!m || !t) return fail(NB_EINVAL, "NULL argument");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  *t = nb_tuning{};
  t->block_threads = m->bs;
  t->blocks = m->nblocks;
  t->row_cost = m->tune_row_cost;
  return NB_OK;
}

// --- the tuning cache: a JSON object mapping a shape key to its winning launch shape,
// {"<key>": {"block_threads": 512, "blocks": 256, "row_cost": 1, "ms": 0.93, "trial_steps": 10}, ...}
struct TuneRec {
  int bs = 0, blocks = 0;
  double row_cost = 1.0, ms = 0.0;
  long long trial = 0;
};

// Key: device (architecture and CU count) and the model's shape -- flavours, N_E, N_u,
// azimuthal bins, species rows, precision, block limit; for batches the model count, rows,
// beams and an FNV-1a hash of every member's (N_E, N_u).
static int tuning_key(const nb_model* m, std::string* key) {
  hipDeviceProp_t prop;
  NB_HIP(hipGetDeviceProperties(&prop, m->device));
  std::string arch;
  for (const char* c = prop.gcnArchName; *c && arch.size() < 64; ++c)
    if (*c != '"' && *c != '\\' && (unsigned char)*c >= 0x20 && (unsigned char)*c < 0x7f) arch += *c;
  const Sub& s = m->subs[0];
  char buf[320];
  snprintf(buf, sizeof buf, "%s/cu%d/nf%d/ne%lld/nu%lld/nphi%lld/ns%d/%s/maxb%d", arch.c_str(), m->cus, m->nf,
           s.NE, s.NU, s.NP, s.NS, state_fp32(m) ? "fp32state" : "fp64", (int)m->p.max_blocks);
  *key = buf;
  if (m->batch) {
    unsigned long long h = 1469598103934665603ull;
    for (const Sub& x : m->subs)
      for (long long v : {x.NE, x.NU})
        for (int b = 0; b < 8; ++b) h = (h ^ (unsigned long long)((v >> (8 * b)) & 0xff)) * 1099511628211ull;
    snprintf(buf, sizeof buf, "/batch%d/rows%lld/beams%lld/h%016llx", m->nmodels, m->rows, m->nb, h);
    *key += buf;
  }
  return NB_OK;
}

class JsonIn {
 public:
  explicit JsonIn(const std::string& t) : t_(t) {}
  void ws() {
    while (i_ < t_.size() && (t_[i_] == ' ' || t_[i_] == '\t' || t_[i_] == '\n' || t_[i_] == '\r')) ++i_;
  }
  bool lit(char c) {
    ws();
    if (i_ < t_.size() && t_[i_] == c) {
      ++i_;
      return true;
    }
    return false;
  }
  bool at_end() {
    ws();
    return i_ == t_.size();
  }
  bool str(std::string& out) {
    if (!lit('"')) return false;
    out.clear();
    while (i_ < t_.size() && t_[i_] != '"') {
      char c = t_[i_++];
      if (c == '\\') {
        if (i_ >= t_.size()) return false;
        const char e = t_[i_++];
        if (e == '"' || e == '\\' || e == '/') c = e;
        else if (e == 'n') c = '\n';
        else if (e == 't') c = '\t';
        else if (e == 'r') c = '\r';
        else if (e == 'b') c = '\b';
        else if (e == 'f') c = '\f';
        else if (e == 'u') {   // \u00XX only (keys are ASCII)
          if (i_ + 4 > t_.size()) return false;
          unsigned v = 0;
          for (int k = 0; k < 4; ++k) {
            const char h = t_[i_++];
            int d = -1;
            if (h >= '0' && h <= '9') d = h - '0';
            else if (h >= 'a' && h <= 'f') d = h - 'a' + 10;
            else if (h >= 'A' && h <= 'F') d = h - 'A' + 10;
            if (d < 0) return false;
            v = v * 16 + (unsigned)d;
          }
          if (v >= 0x80) return false;
          c = (char)v;
        } else {
          return false;
        }
      }
      out += c;
    }
    return lit('"');
  }
  bool num(double& v) {
    ws();
    const char* b = t_.c_str() + i_;
    char* e = nullptr;
    v = std::strtod(b, &e);
    if (e == b) return false;
    i_ += (size_t)(e - b);
    return true;
  }
  // any value (unknown fields): string, number, literal, or nested object/array
  bool skip() {
    ws();
    if (i_ >= t_.size()) return false;
    const char c = t_[i_];
    if (c == '"') {
      std::string tmp;
      return str(tmp);
    }
    if (c == '{' || c == '[') {
      const char close = (c == '{') ? '}' : ']';
      ++i_;
      if (lit(close)) return true;
      do {
        if (c == '{') {
          std::string k;
          if (!str(k) || !lit(':')) return false;
        }
        if (!skip()) return false;
      } while (lit(','));
      return lit(close);
    }
    for (const char* w : {"true", "false", "null"})
      if (t_.compare(i_, std::strlen(w), w) == 0) {
        i_ += std::strlen(w);
        return true;
      }
    double v;
    return num(v);
  }

 private:
  const std::string& t_;
  size_t i_ = 0;
};

// Read the cache (a missing file is an empty cache).  NB_EIO if it cannot be read or is
// not a tuning cache; it is then left as it is.
static int read_cache(const char* path, std::map<std::string, TuneRec>* recs) {
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    if (errno == ENOENT) return NB_OK;
    return fail(NB_EIO, "tuning cache %s: %s", path, std::strerror(errno));
  }
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  const bool err = std::ferror(f) != 0;
  std::fclose(f);
  if (err) return fail(NB_EIO, "tuning cache %s: read error", path);
  if (text.size() > (64u << 20)) return fail(NB_EIO, "tuning cache %s: larger than 64 MiB", path);
  JsonIn in(text);
  if (in.at_end()) return NB_OK;   // empty file
  if (!in.lit('{')) return fail(NB_EIO, "tuning cache %s: not a JSON object", path);
  if (!in.lit('}')) {
    do {
      std::string key;
      if (!in.str(key) || !in.lit(':') || !in.lit('{'))
        return fail(NB_EIO, "tuning cache %s: malformed entry", path);
      TuneRec r;
      bool have_bs = false, have_blocks = false;
      if (!in.lit('}')) {
        do {
          std::string f2;
          if (!in.str(f2) || !in.lit(':')) return fail(NB_EIO, "tuning cache %s: malformed field", path);
          double v = 0.0;
          const bool known = f2 == "block_threads" || f2 == "blocks" || f2 == "row_cost" || f2 == "ms" ||
                             f2 == "trial_steps";
          if (known ? !in.num(v) : !in.skip())
            return fail(NB_EIO, "tuning cache %s: bad value of %s", path, f2.c_str());
          if (f2 == "block_threads") { r.bs = (int)v; have_bs = true; }
          else if (f2 == "blocks") { r.blocks = (int)v; have_blocks = true; }
          else if (f2 == "row_cost") r.row_cost = v;
          else if (f2 == "ms") r.ms = v;
          else if (f2 == "trial_steps") r.trial = (long long)v;
        } while (in.lit(','));
        if (!in.lit('}')) return fail(NB_EIO, "tuning cache %s: unterminated entry", path);
      }
      if (have_bs && have_blocks) (*recs)[key] = r;
    } while (in.lit(','));
    if (!in.lit('}')) return fail(NB_EIO, "tuning cache %s: unterminated object", path);
  }
  if (!in.at_end()) return fail(NB_EIO, "tuning cache %s: trailing characters", path);
  return NB_OK;
}

// Write the cache: a temporary file beside it, then renamed over it (readers see the old
// or the new file, never a partial one).
static int write_cache(const char* path, const std::map<std::string, TuneRec>& recs) {
  std::string out = "{\n";
  size_t i = 0;
  for (const auto& kv : recs) {
    std::string k;
    for (char c : kv.first) {
      if (c == '"' || c == '\\') k += '\\';
      k += c;
    }
    char buf[256];
    snprintf(buf, sizeof buf,
             "\": {\"block_threads\": %d, \"blocks\": %d, \"row_cost\": %.17g, \"ms\": %.17g, \"trial_steps\": %lld}",
             kv.second.bs, kv.second.blocks, kv.second.row_cost, kv.second.ms, kv.second.trial);
    out += "  \"" + k + buf + (++i < recs.size() ? ",\n" : "\n");
  }
  out += "}\n";
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(NB_EIO, "tuning cache %s: %s", tmp.c_str(), std::strerror(errno));
  const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed || std::rename(tmp.c_str(), path) != 0) {
    const int e = errno;
    std::remove(tmp.c_str());
    return fail(NB_EIO, "tuning cache %s: write failed (%s)", path, std::strerror(e));
  }
  return NB_OK;
}

// Times trial_steps steps from the initial state (best of two runs, after a one-step
// warm-up launch) for every candidate shape: 512 and 256 threads per block, each at the
// full resident grid, 3/4 and 1/2 of it; for batches each with row costs 0.25, 1 and 3
// chunks.  Keeps the fastest, then resets the model.
extern "C" int nb_autotune(nb_model* m, int32_t trial_steps, const char* cache_path, nb_tuning* out) {
  if (!m) return fail(NB_EINVAL, "model is NULL");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (trial_steps < 1) return fail(NB_EINVAL, "trial_steps must be >= 1");
  if (capturing(m->stream)) return fail(NB_EINVAL, "the autotuner cannot run under capture");
  drop_graph(m);
  std::map<std::string, TuneRec> recs;
  std::string key;
  const bool use_cache = cache_path && *cache_path;
  if (use_cache) {
    int rc = tuning_key(m, &key);
    if (!rc) rc = read_cache(cache_path, &recs);
    if (rc) return rc;
    const auto it = recs.find(key);
    if (it != recs.end() && it->second.blocks >= 1 &&
        check_shape(m, it->second.bs, it->second.blocks, it->second.row_cost) == NB_OK) {
      const TuneRec& r = it->second;
      rc = apply_shape(m, r.bs, r.blocks, m->batch ? r.row_cost : m->tune_row_cost);
      if (!rc) rc = nb_reset(m);
      if (rc) return rc;
      if (out) {
        nb_get_tuning(m, out);
        out->ms = r.ms;
        out->from_cache = 1;
        out->candidates = 0;
      }
      return NB_OK;
    }
  }
  struct Cand {
    int bs, blocks;
    double cost;
  };
  std::vector<Cand> cands;
  const std::vector<double> costs = m->batch ? std::vector<double>{0.25, 1.0, 3.0}
                                             : std::vector<double>{m->tune_row_cost};
  for (int bs : {kBlock, kBlockSmall}) {
    if (capacity(m, bs) < 1) continue;
    const int full = blocks_for(m, bs, 0);
    std::vector<int> bl = {full};
    if (full >= 8) {
      bl.push_back(full * 3 / 4);
      bl.push_back(full / 2);
    }
    for (int b : bl)
      for (double c : costs) cands.push_back({bs, b, c});
  }
  hipEvent_t e0, e1;
  NB_HIP(hipEventCreate(&e0));
  NB_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  Cand pick = cands[0];
  int rc = NB_OK;
  const long long steps = std::min<long long>(trial_steps, m->p.n_steps);
  for (const Cand& c : cands) {
    if ((rc = apply_shape(m, c.bs, c.blocks, c.cost))) break;
    if ((rc = nb_reset(m)) || (rc = nb_step(m, 1))) break;      // warm-up launch
    float mine = 1e30f;
    for (int rep = 0; rep < 2 && !rc; ++rep) {
      if ((rc = nb_reset(m))) break;
      hipError_t e = hipEventRecord(e0, m->stream);
      if (e == hipSuccess && !(rc = nb_step(m, steps))) {
        e = hipEventRecord(e1, m->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) mine = std::min(mine, ms);
      }
      if (e != hipSuccess && !rc) rc = fail(NB_EHIP, "autotune timing: %s", hipGetErrorString(e));
    }
    if (rc) break;
    if (mine < best) {
      best = mine;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int r2 = apply_shape(m, pick.bs, pick.blocks, pick.cost);
  if (!rc) rc = r2;
  int r3 = nb_reset(m);
  if (!rc) rc = r3;
  if (rc) return rc;
  if (use_cache) {
    TuneRec r;
    r.bs = pick.bs;
    r.blocks = pick.blocks;
    r.row_cost = pick.cost;
    r.ms = best;
    r.trial = steps;
    recs[key] = r;
    rc = write_cache(cache_path, recs);
    if (rc) return rc;
  }
  if (out) {
    nb_get_tuning(m, out);
    out->ms = best;
    out->from_cache = 0;
    out->candidates = (int32_t)cands.size();
  }
  return NB_OK;
}

extern "C" int nb_read_pee(const nb_model* m, double* dev_out) {
  if (!m || !dev_out) return fail(NB_EINVAL, "NULL argument");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  void* X = m->ws + m->off_X;
  long long nb_ = m->nb, plane = m->plane;
  int nsc = m->nsc;
  void* args[] = {&X, &nb_, &plane, &nsc, &dev_out};
  int rc = launch_1d(state_fp32(m) ? (const void*)&k_read_pee<float> : (const void*)&k_read_pee<double>,
                     m->nb, args, m->stream);
  if (rc) return rc;
  if (!capturing(m->stream)) NB_HIP(hipStreamSynchronize(m->stream));
  return NB_OK;
}

static int xfer(nb_model* m, double* buf, int dir) {
  void* X = m->ws + m->off_X;
  long long nb_ = m->nb, plane = m->plane;
  int nsc = m->nsc;
  void* args[] = {&X, &nb_, &plane, &nsc, &buf, &dir};
  return launch_1d(state_fp32(m) ? (const void*)&k_state_xfer<float> : (const void*)&k_state_xfer<double>,
                   m->nb, args, m->stream);
}

// Host <-> state planes without a device buffer: FP64 states as one strided copy of the
// nsc planes (pitch plane -> nb beams); FP32 states through a host buffer, converted on the
// host (double -> float rounds to nearest, as the kernels do).
static int host_xfer(nb_model* m, double* host, int dir) {
  const size_t es = state_fp32(m) ? sizeof(float) : sizeof(double);
  char* X = m->ws + m->off_X;
  const size_t nbb = (size_t)m->nb, rows = (size_t)m->nsc;
  std::vector<float> f;
  void* hbuf = host;
  if (es == sizeof(float)) {
    f.resize(nbb * rows);
    if (dir == 1)
      for (size_t i = 0; i < f.size(); ++i) f[i] = (float)host[i];
    hbuf = f.data();
  }
  hipError_t e = (dir == 0)
                     ? hipMemcpy2DAsync(hbuf, es * nbb, X, es * (size_t)m->plane, es * nbb, rows,
                                        hipMemcpyDeviceToHost, m->stream)
                     : hipMemcpy2DAsync(X, es * (size_t)m->plane, hbuf, es * nbb, es * nbb, rows,
                                        hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return fail(NB_EHIP, "state copy: %s", hipGetErrorString(e));
  if (es == sizeof(float) && dir == 0)
    for (size_t i = 0; i < f.size(); ++i) host[i] = (double)f[i];
  return NB_OK;
}

extern "C" int nb_get_state(const nb_model* mc, double* dst, int on_device) {
  nb_model* m = const_cast<nb_model*>(mc);
  if (!m || !dst) return fail(NB_EINVAL, "NULL argument");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (capturing(m->stream)) return fail(NB_EINVAL, "state exchange cannot be captured");
  if (!on_device) return host_xfer(m, dst, 0);
  int rc = xfer(m, dst, 0);
  if (rc) return rc;
  NB_HIP(hipStreamSynchronize(m->stream));
  return NB_OK;
}

extern "C" int nb_set_state(nb_model* m, const double* src, int64_t step, int on_device) {
  if (!m || !src) return fail(NB_EINVAL, "NULL argument");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (step < 0 || step > m->p.n_steps) return fail(NB_EINVAL, "step out of range");
  if (capturing(m->stream)) return fail(NB_EINVAL, "state exchange cannot be captured");
  int rc = on_device ? xfer(m, const_cast<double*>(src), 1) : host_xfer(m, const_cast<double*>(src), 1);
  if (rc) return rc;
  rc = set_device_step(m, step);
  if (rc) return rc;
  NB_HIP(hipStreamSynchronize(m->stream));
  m->step = step;
  return NB_OK;
}

extern "C" int nb_adjoint(nb_model* m, const double* dev_dl_dpee, double* grad_out, int32_t ckpt_every,
                          double* dev_state_bar) {
  if (!m || !grad_out) return fail(NB_EINVAL, "NULL model or gradient output");
  if (!m->ws) return fail(NB_EUNBOUND, "no workspace bound");
  if (!adjoint_enabled(m))
    return fail(NB_EINVAL, "the adjoint needs a single two-flavour model created with adjoint_ckpt > 0");
  if (ckpt_every < 0) return fail(NB_EINVAL, "ckpt_every must be >= 0");
  if (capturing(m->stream)) return fail(NB_EINVAL, "the adjoint cannot be captured into a graph");
  if (!m->adj_bpt) return fail(NB_EUNBOUND, "adjoint launch shape not set (bind the model)");
  const long long K = ckpt_every > 0 ? ckpt_every : m->p.adjoint_ckpt;
  const long long n0 = m->step, N = m->p.n_steps, ns = N - n0;
  const long long nseg = (ns + K - 1) / K;
  if (nseg + std::min(K, ns) > adjoint_slots(m))
    return fail(NB_EINVAL, "checkpoint period %lld needs %lld state slots; the workspace holds %lld", K,
                nseg + std::min(K, ns), adjoint_slots(m));
  const size_t pl3 = (size_t)3 * m->plane;
  double* ck = (double*)(m->ws + m->off_adj);
  double* tape = ck + (size_t)nseg * pl3;
  // forward pass: checkpoint at the start of every segment, every stage's moments recorded
  m->jhist = (double*)(m->ws + m->off_jhist);
  for (long long sg = 0; sg < nseg; ++sg) {
    const hipError_t e = hipMemcpyAsync(ck + sg * pl3, m->ws + m->off_X, sizeof(double) * pl3,
                                        hipMemcpyDeviceToDevice, m->stream);
    if (e != hipSuccess) {
      m->jhist = nullptr;
      return fail(NB_EHIP, "checkpoint copy: %s", hipGetErrorString(e));
    }
    const int rc = advance(m, std::min(K, ns - sg * K));
    if (rc) {
      m->jhist = nullptr;
      return rc;
    }
  }
  m->jhist = nullptr;
  // reverse pass
  unsigned int* sync = (unsigned int*)(m->ws + m->off_sync);
  int rc0 = zero_sync(m, 1);
  if (rc0) return rc0;
  const Sub& s = m->subs[0];
  AdjArgs a{};
  a.tab = (const double*)(m->ws + m->off_tab);
  a.dtab = (const double*)(m->ws + m->off_dtab);
  a.Jhist = (const double*)(m->ws + m->off_jhist);
  a.ck = ck;
  a.tape = tape;
  a.cot = dev_dl_dpee;
  a.cot_const = ((s.p.e_max_mev - s.p.e_min_mev) / (double)s.NE) / (double)s.NU;
  a.state_bar = dev_state_bar;
  a.spill = (double*)(m->ws + m->off_spill);
  a.out = (double*)(m->ws + m->off_aout);
  a.sync = sync;
  a.plane = m->plane;
  a.nb = m->nb;
  a.NE = (int)s.NE;
  a.NU = (int)s.NU;
  a.n0 = n0;
  a.nsteps = ns;
  a.ckpt = K;
  a.nseg = nseg;
  a.rs = m->p.r_start_km;
  a.h = s.h;
  a.R = m->p.r_nu_km;
  a.lam0 = s.lam0;
  a.s2gf = potential_per_density();
  a.ne_power = m->p.ne_power;
  a.renorm = m->p.renorm;
  a.timeout_ticks = m->ticks_per_s * 20ull;
  a.cancel = m->cancel_dev;
  void* args[] = {&a};
  const void* fn = m->adj_bpt == 1 ? (const void*)&k_adjoint2<1>
                 : m->adj_bpt == 2 ? (const void*)&k_adjoint2<2>
                 : m->adj_bpt == 4 ? (const void*)&k_adjoint2<4>
                                   : (const void*)&k_adjoint2<0>;
  const hipError_t e = hipLaunchKernel(fn, dim3(m->adj_blocks), dim3(kBlock), args, 0, m->stream);
  if (e != hipSuccess) return fail(NB_EHIP, "adjoint launch: %s", hipGetErrorString(e));
  const long long before = m->step;
  int rc = check_status(m);
  if (rc) return rc;
  if (m->step != before) return fail(NB_EHIP, "device step counter moved during the reverse pass");
  double* host = (double*)(m->pinned + 8);
  NB_HIP(hipMemcpyAsync(host, a.out, sizeof(double) * 5, hipMemcpyDeviceToHost, m->stream));
  NB_HIP(hipStreamSynchronize(m->stream));
  for (int i = 0; i < 5; ++i) {
    grad_out[i] = host[i];
    if (!std::isfinite(host[i])) return fail(NB_ENUMERIC, "non-finite gradient component %d", i);
  }
  return NB_OK;
}

extern "C" int nb_host_tables(const nb_model* m, double* out, int64_t cap) {
  if (!m || !out) return fail(NB_EINVAL, "NULL argument");
  if (m->batch) return fail(NB_EINVAL, "host tables are reported for single models");
  const Sub& s = m->subs[0];
  const int nv = (m->nf == 2) ? 2 : 6;
  const int rows = (m->nf == 2) ? 2 : kVacRows3;   // table rows before the weights
  const long long NE = s.NE;
  const long long need = NE + (long long)s.NS * NE + nv * NE + 7;
  if (cap < need) return fail(NB_EINVAL, "output too small (%lld needed)", need);
  long long o = 0;
  for (long long k = 0; k < NE; ++k) out[o++] = s.E[k];
  for (int sp = 0; sp < s.NS; ++sp)
    for (long long k = 0; k < NE; ++k) out[o++] = s.tab[(size_t)(rows + sp) * NE + k];
  for (long long k = 0; k < NE; ++k)
    for (int q = 0; q < nv; ++q) out[o++] = s.tab[(size_t)q * NE + k];
  out[o++] = s.lam0;
  out[o++] = s.kappa0;
  out[o++] = s.h;
  out[o++] = s.p2e1;
  out[o++] = s.p2e0;
  out[o++] = s.e1;
  out[o++] = s.e0;
  return NB_OK;
}
