/*
 * nubulb.h -- C-ABI of the MI355X bulb-model radial stepper.
 *
 * The library advances the flavour state of every (species, emission bin, energy bin)
 * beam of the neutrino bulb model (paper, Sec. 2) along the radius r.  One radial step is
 * a Lie-group Runge-Kutta step of order 4 (classical RK4 tableau on the unitary group,
 * Munthe-Kaas 1999) whose exponential map is the exact one-step propagator exp(-i H dl),
 * dl = dr/cos(theta) (Eq. U), and whose Hamiltonian
 *     H = H_vac(E) + H_mat(r) + H_nunu(theta; r)                       (Eq. eom)
 * is rebuilt at every stage from two moments of all beams, J0 = sum g rho~/cos(theta')
 * and J1 = sum g rho~ (Eqs. Hnu and F), summed exactly in fixed point (the extended model
 * adds J_sc and J_ss, the sin(theta) cos(phi) and sin(theta) sin(phi) moments of Eq. F, and
 * H_nunu gains - sin(theta) (cos(phi) J_sc + sin(phi) J_ss)).  Antineutrinos
 * evolve with H_vac - H_mat - H_nunu^* (Eq. eom).  Every beam starts in its flavour
 * eigenstate at r_start (Sec. 3.4).
 *
 * Conventions for every entry point:
 *   - return value: NB_OK (0) or a negative NB_E* code; nb_last_error() then holds a
 *     message for the calling thread.  No C++ exception crosses this boundary.
 *   - ownership: the caller owns every buffer (device workspace, outputs).  The library
 *     owns only the opaque nb_model host object, freed by nb_model_destroy.
 *   - device memory: all device work uses the workspace bound with nb_bind; nb_step,
 *     nb_run, nb_read_pee and nb_adjoint allocate nothing (the adjoint's checkpoints and
 *     tape are part of the workspace when adjoint_ckpt > 0).
 *   - streams: all device work is enqueued on the stream given to nb_bind.  Calls return
 *     after checking the kernels' status word, i.e. after the stream has drained, unless
 *     the stream is being captured into a HIP graph (then they return at once).
 *   - beam index b = ((s * n_u + j) * n_phi + p) * n_energy + k, with species s
 *     (0 = nu_e-born, 1 = anti-nu_e-born; with track_all s = anti * n_flavor + flavour of
 *     birth), emission bin j, azimuthal bin p (n_phi = 1 and p = 0 for the bulb model) and
 *     energy bin k; energy is innermost.
 *   - layouts of device buffers are plain arrays of double in that beam order.
 *   - errors are checked before any device work is enqueued.
 */
#ifndef NUBULB_H
#define NUBULB_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NB_OK = 0,
  NB_EINVAL = -1,      /* invalid parameter or argument */
  NB_EUNBOUND = -2,    /* no workspace bound yet */
  NB_EWORKSPACE = -3,  /* workspace too small or misaligned (256 B) */
  NB_EHIP = -4,        /* a HIP runtime call failed (no device, launch failure, ...) */
  NB_ENUMERIC = -5,    /* a moment contribution left the fixed-point range (NaN/overflow), or
                          a renormalised state had |psi|^2 (|P|^2) off 1 by more than 1e-8
                          (FP32 states: 1e-5) before the renormalisation */
  NB_ETIMEOUT = -6,    /* a grid barrier did not complete within its time limit (20 s), or the
                          host cancelled the model's launches (nb_cancel) */
  NB_ESTEP = -7,       /* adaptive step control failed (step length underflow or attempt limit) */
  NB_EIO = -8          /* the autotuner's cache file could not be read, parsed or written */
};

enum { NB_FP64 = 0, NB_FP32_STATE = 1 };

/* Model parameters (paper, Sec. 2 and Sec. 3.2).  Lengths in km, energies in MeV. */
typedef struct {
  int32_t n_flavor;     /* 2 (e, x) or 3 (e, mu, tau) */
  int32_t n_energy;     /* N_E bins of equal width over [e_min_mev, e_max_mev], midpoints */
  int32_t n_u;          /* N_u bins of equal width in u = sin^2(theta_R) over [0,1], midpoints */
  int32_t ne_power;     /* n_e(r) = n0_cm3 (R/r)^ne_power; 3 for the bulb, 0..8 allowed */
  int32_t precision;    /* NB_FP64, or NB_FP32_STATE (3 flavours: state stored in FP32;
                           at most 2^30 - 64 beams, NB_EINVAL beyond) */
  int32_t renorm;       /* 1: renormalise every beam after every step (0: tests only); the
                           factor is 1.5 - n^2/2, exact to rounding for the near-unit norms a
                           step leaves (initial states must have unit norm) */
  int32_t adjoint_ckpt; /* >0: reserve workspace for nb_adjoint with this checkpoint period */
  int32_t max_blocks;   /* 0: as many blocks as fit on the device; else an upper bound */
  int64_t n_steps;      /* radial steps from r_start_km to r_end_km */
  double e_min_mev, e_max_mev;
  double r_nu_km;       /* neutrinosphere radius R */
  double r_start_km, r_end_km;
  double lum_erg_s[3];  /* luminosities of nu_e, anti-nu_e, nu_x (= each heavy flavour) */
  double temp_mev[3];   /* Fermi-Dirac temperatures, zero chemical potential */
  double dm2_ev2[2];    /* 2f: [0] = dm^2.  3f: dm^2_21, dm^2_31 */
  double theta[3];      /* 2f: [0] = theta_v.  3f: theta_12, theta_13, theta_23 */
  double delta_cp;      /* must be 0 (real mixing matrix) */
  double n0_cm3;        /* electron density scale */
  int32_t adaptive;     /* 1: reserve workspace for nb_run_adaptive (single FP64 models) */
  int32_t n_phi;        /* 0: the bulb model.  >= 1: the extended bulb model (Sec. 2, the
                           replacements of Eq. int-v) with n_phi azimuthal bins of equal
                           width over [0, 2 pi); single FP64 models, fixed steps */
  int32_t track_all;    /* 0: track the nu_e- and anti-nu_e-born beams (heavy-flavour-born
                           states follow from unitarity); 1: track every initially populated
                           flavour explicitly (the paper's four particles, six for three
                           flavours); single models without adjoint */
  int32_t reserved;     /* must be 0 */
  double lum_xbar_erg_s;/* anti-nu_x (each heavy antiflavour) luminosity and temperature; */
  double temp_xbar_mev; /* temp_xbar_mev = 0: the nu_x values lum_erg_s[2], temp_mev[2] */
} nb_params;

typedef struct nb_model nb_model;

/* Create a model: validates p and builds the host tables (E bins, spectra, weights,
 * vacuum Hamiltonians, fixed-point scales).  No device work.  *out is NULL on error. */
int nb_model_create(const nb_params *p, nb_model **out);
/* Create a batch of n_models independent 2-flavour models advanced together (all must
 * share n_steps, r_start_km and r_end_km).  Beams of model m follow those of m-1. */
int nb_batch_create(const nb_params *p, int32_t n_models, nb_model **out);
void nb_model_destroy(nb_model *m);

int64_t nb_n_beams(const nb_model *m);      /* all models of a batch */
int32_t nb_n_models(const nb_model *m);
int32_t nb_state_comps(const nb_model *m);  /* 3 (2f Bloch vector) or 6 (3f wavefunction) */
/* Offsets of each model's beams in beam-indexed outputs: off[0..n_models]. */
int nb_pee_offsets(const nb_model *m, int64_t *off);
/* Bytes of device workspace the model needs (256-byte aligned start required). */
size_t nb_workspace_bytes(const nb_model *m);
/* Bind caller-owned device memory and a HIP stream (hipStream_t, may be NULL) on the
 * current device: measure the resident capacity of the stepping kernels there, upload the
 * tables of Sec. 3.2 (energy bins, emission weights of Eqs. Hnu and F, vacuum
 * Hamiltonians of Sec. 2) on that stream and reset the state (as nb_reset).  A model may be
 * bound again (another workspace or stream); that drops its graph.  NB_EWORKSPACE if
 * bytes < nb_workspace_bytes or dev_ws is not 256-byte aligned. */
int nb_bind(nb_model *m, void *dev_ws, size_t bytes, void *hip_stream);
/* Every beam back to its initial flavour eigenstate at r_start (Sec. 3.4); step = 0. */
int nb_reset(nb_model *m);
/* Advance n radial steps of the fixed grid r_k = r_start + k (r_end - r_start)/n_steps
 * (bounded by n_steps - current step): each step is the RKMK4 step of Eq. U with the
 * Hamiltonian of Eq. eom rebuilt at every stage from the moments of Eqs. Hnu and F (see
 * the preamble).  One persistent launch per chunk of steps (so that the barrier
 * epochs of a launch stay within 32 bits); returns after the stream has drained and the
 * kernels' status word was checked.  NB_ENUMERIC: a moment contribution left its
 * fixed-point range (NaN or overflow), or a state's norm was off 1 by more than a unitary
 * step's rounding explains (renorm = 1); NB_ETIMEOUT: a grid
 * barrier timed out or the model was cancelled -- in both cases the state is undefined
 * until nb_reset or nb_set_state, except after a cancel that took effect before the launch
 * started, which leaves state and step as they were. */
int nb_step(nb_model *m, int64_t n);
/* Advance to r_end_km (nb_step of the remaining steps). */
int nb_run(nb_model *m);
int64_t nb_step_index(const nb_model *m);
/* For callers that cannot allocate device memory or use the workspace's scratch (code
 * under graph capture, tight serving loops, harnesses that forbid allocation): nb_step
 * with the scratch of the stepping launches -- the barrier and tagged reduction words and,
 * for batches, the moment accumulators -- taken from a static device array of the library
 * instead of the bound workspace (3.3 MB per device, held until the process ends).  Same
 * kernels and the same bits as nb_step; the model's state, tables and step counter stay
 * in its workspace.  Allocates nothing.  Limits: at most 1024 models in a batch and 2048
 * blocks per launch (every launch shape nb_bind picks fits), NB_EINVAL beyond.  Every call
 * on one device shares that device's array and clears it first, so calls that overlap on
 * one device (other host threads, other streams) race and must be serialised by the
 * caller.  Errors as nb_step. */
int nb_step_static(nb_model *m, int64_t n);
/* Survival probability Re(rho_ee) of every beam (paper's P_ee, Sec. 3.5) into the
 * caller's device array dev_out[nb_n_beams]. */
int nb_read_pee(const nb_model *m, double *dev_out);
/* State exchange as FP64 planes [comp][beam] (2f: P_x, P_y, P_z; 3f: Re/Im psi_e,
 * psi_mu, psi_tau).  on_device: 1 if dst/src is device memory, 0 if host memory (pageable
 * or pinned; FP32 states are converted on the host).  Allocates no device memory.
 * nb_set_state also sets the step index (0 <= step <= n_steps). */
int nb_get_state(const nb_model *m, double *dst, int on_device);
int nb_set_state(nb_model *m, const double *src, int64_t step, int on_device);

/* Mixed precision (3 flavours, precision = NB_FP32_STATE): the state is stored in FP32; the
 * moment sums and the renormalisation of each updated state are FP64.  The per-beam stage
 * arithmetic (generators, commutators, exponentials) is FP32 from the returned step on,
 * where an a-priori bound shows every beam's per-step rotation angle below one radian, and
 * FP64 before it (nearer the neutrinosphere FP32 cannot hold the per-step phase).  Returns
 * that step (n_steps if FP32 arithmetic is never used), or -1 for other models. */
int64_t nb_mixed_fp32_step(const nb_model *m);

/* HIP graph of one stepping launch: nb_graph_capture records "advance n_steps from the
 * device step counter" (n_steps >= 1) on the bound stream (which must not be the NULL
 * stream) into a graph held by the model; nb_graph_launch replays it and checks the
 * status word.  Every replay continues from where the previous one stopped and stops at
 * r_end.  Rebinding, changing the launch shape (nb_autotune, nb_set_tuning) or destroying
 * the model drops the graph.  Every persistent launch of the library (eager or in a graph)
 * is an ordinary kernel launch whose grid never exceeds the resident capacity measured at
 * nb_bind, which makes progress while all its blocks are resident at once: nb_graph_launch
 * also refuses (NB_EINVAL) a recorded grid above the capacity the device reports at the
 * time of the launch, and work that other streams run meanwhile can still stall a launch
 * -- the barrier waits then end at their 20 s limit or at nb_cancel with NB_ETIMEOUT. */
int nb_graph_capture(nb_model *m, int64_t n_steps);
int nb_graph_launch(nb_model *m);

/* Cancel: while on != 0, every persistent launch of the model (stepping, graph replays,
 * adaptive, adjoint) that starts returns at once without touching the state, and one that
 * is waiting in a grid barrier gives up within about a millisecond; both end in
 * NB_ETIMEOUT ("cancelled by the host").  on = 0 lets launches run again.  The flag is a
 * word of fine-grained pinned host memory: this call may come from any host thread at any
 * time, including while another thread is inside nb_step or nb_graph_launch of the model.
 * Requires a bound model. */
int nb_cancel(nb_model *m, int32_t on);

/* Launch shape of the fixed-step kernels (single models and batches; the adaptive and
 * adjoint kernels keep their own).  A beam's arithmetic does not depend on it, and the
 * moments are exact integer sums, so every shape gives the same bits.  Default (until
 * nb_autotune or nb_set_tuning): 256 threads per block for two flavours, 512 for three, at
 * the full resident grid. */
typedef struct {
  int32_t block_threads;  /* threads per block: 512 (8 wavefronts) or 256 (4) */
  int32_t blocks;         /* block cap of a launch (nb_set_tuning: 0 = the resident capacity);
                             a launch uses at most one wavefront per row */
  double row_cost;        /* batches: per-row overhead, in 64-lane chunks, of the cost model
                             that splits the rows among wavefronts (default 1) */
  double ms;              /* nb_autotune: time of the winning trial (on a cache hit: as stored) */
  int32_t from_cache;     /* nb_autotune: 1 if the shape came from the cache file */
  int32_t candidates;     /* nb_autotune: launch shapes timed (0 on a cache hit) */
} nb_tuning;

/* Autotuner.  With cache_path (a JSON file; NULL or "": no cache) it first looks up the
 * key of this device and shape -- architecture, CU count, flavours, N_E, N_u, azimuthal
 * bins, species rows, precision, max_blocks, and for batches the model count, rows, beams
 * and a hash of every member's (N_E, N_u) -- and applies a stored shape without timing
 * anything.  Otherwise it times trial_steps steps from the initial state (best of two,
 * HIP events) for every candidate: 512 and 256 threads per block, each at the full
 * resident grid, 3/4 and 1/2 of it, and for batches row costs 0.25, 1 and 3; keeps the
 * fastest and adds it to the cache (written to a temporary file, then renamed over it).
 * The model is then reset to step 0.  *out (may be NULL) receives the shape.  NB_EIO if
 * the cache cannot be read, is not such a JSON object, or cannot be written (a malformed
 * file is left as it is); not capturable. */
int nb_autotune(nb_model *m, int32_t trial_steps, const char *cache_path, nb_tuning *out);
/* Apply a launch shape (block_threads, blocks, row_cost; the other fields are ignored).
 * NB_EINVAL if the stepping kernels cannot be resident at that block size or blocks
 * exceeds the resident capacity.  Keeps the state and the step index. */
int nb_set_tuning(nb_model *m, const nb_tuning *t);
/* The shape in use: block_threads, blocks of a launch, row_cost; other fields zero. */
int nb_get_tuning(const nb_model *m, nb_tuning *t);

/* Reverse-mode adjoint of the radial integration (2 flavours, FP64, single model created
 * with adjoint_ckpt > 0).  The gradients are those of the final survival probabilities
 * (Sec. 3.5) with respect to the luminosities, the vacuum mixing angle (Sec. 2) and the
 * electron density scale of n_e(r) (Sec. 3.2), for L = sum_b dL/dPee_b Pee_b at r_end.
 * Runs forward from the current state and step to r_end, keeping the state every
 * ckpt_every steps (0: the model's adjoint_ckpt) and recording every stage's moments,
 * then backwards one segment at a time, each segment recomputed from its checkpoint.
 *   dev_dl_dpee    [nb_n_beams] device, dL/dPee per beam; NULL: dE/N_u for every beam (the
 *                  energy-integrated, angle-averaged P_ee of both species).
 *   grad_out[5]    host, dL/d{L_e, L_ebar, L_x (erg/s), theta_v (rad), n0 (cm^-3)}.
 *   dev_state_bar  NULL, or [3][nb_n_beams] device: dL/d(Bloch vectors at the start step).
 * The period must fit the workspace: ceil(steps/ckpt) + min(ckpt, steps) state slots, no
 * more than ceil(n_steps/adjoint_ckpt) + min(adjoint_ckpt, n_steps).  The model is left at
 * r_end with the forward run's state.  Moment adjoints are summed in FP64 in a fixed
 * order, so results repeat bit for bit.  Not capturable into a graph (it synchronises). */
int nb_adjoint(nb_model *m, const double *dev_dl_dpee, double *grad_out, int32_t ckpt_every,
               double *dev_state_bar);

/* Adaptive step-size control (the paper's solver adapts its radial step, Sec. 3.4).
 * Integrates from r_start to r_end with RKMK4 steps whose length follows an embedded error
 * estimate: E = max over beams of |Theta - F_2|^2, the squared distance between the order-4
 * generator Theta and the generator F_2 of the exponential midpoint rule built from the
 * same stages (3 flavours: traceless part, Frobenius norm), with the low 16 bits of its
 * binary form cleared.  A step of length h is accepted if E <= tol^2; then h doubles (at
 * most to h_max_km; <= 0: no cap) if E <= tol^2/128.  A rejected step is retried from the
 * same state with h/2.  The last step ends exactly at r_end.  The first step length is
 * (r_end - r_start)/n_steps.  Every decision is taken by every block from the same reduced
 * E, so the run is deterministic and matches a serial implementation bit for bit.
 *   Requires a single FP64 model created with adaptive = 1, at step 0 (after nb_bind or
 *   nb_reset).  On success the state is at r_end and the step index is n_steps.
 *   stats (host, may be NULL): accepted and rejected steps, attempts, and the step length
 *   after the last decision.
 *   NB_ESTEP if h falls below 2^-40 of the first step length or max_attempts is exceeded;
 *   the model is then reset to its initial state.
 * Not capturable into a graph (it synchronises to read the step statistics). */
typedef struct {
  int64_t accepted, rejected, attempts;
  double h_last_km;
} nb_adaptive_stats;
int nb_run_adaptive(nb_model *m, double tol, double h_max_km, int64_t max_attempts,
                    nb_adaptive_stats *stats);

/* Host tables (no device work), layout as [E_k | weights[n_species][NE] | vacuum terms |
 * lam0, kappa0, h, 2^-e1, 2^-e0, e1, e0]; vacuum terms are (B_x, B_z) per k for 2f and
 * 6 entries per k (H_ee, H_mm, H_tt, H_em, H_et, H_mt) for 3f.  Single models only. */
int nb_host_tables(const nb_model *m, double *out, int64_t cap);

const char *nb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
