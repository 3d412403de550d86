// nb_internal.h -- layouts shared by the kernels and the host runtime (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

constexpr int kMaxBlocks = 2048;  // upper bound on blocks of one stepping launch (MI355X: 256 CUs
                                  // hold at most 4 blocks of 512 threads each)

// Offsets (in 32-bit words) of the synchronisation words.  Every word that more than one
// block writes or polls sits on a 128-byte line of its own: the abort and status words,
// kFlagCopies copies of the release flag (block b polls copy b % kFlagCopies) and one
// arrival word per block.
constexpr int kLineWords = 32;
constexpr int kFlagCopies = 8;
constexpr int kSyncAbort = 1 * kLineWords;   // set when any block gives up waiting
constexpr int kSyncStatus = 2 * kLineWords;  // bit 0: fixed-point range error, bit 1: barrier timeout,
                                             // bit 2: cancelled by the host, bit 3: renormalisation
                                             // factor far from 1
constexpr int kSyncFlag = 4 * kLineWords;    // [kFlagCopies] lines: epoch + 1 of the last release
constexpr int kSyncArrive = kSyncFlag + kFlagCopies * kLineWords;  // [kMaxBlocks] lines
// Tagged 64-bit words of the moment reductions (every word carries the barrier epoch it
// belongs to, so no separate arrival or release word is needed): kFlagCopies copies of
// reduced moments (the adjoint's sums; block b reads copy b % kFlagCopies), kTagLines lines
// each; then block partials, one slot of kTagLines lines per block, in two regions used by
// the stepping kernels at even and odd epochs (the adjoint uses the first).
constexpr int kTagLines = 4;
constexpr int kSyncJTag = kSyncArrive + kMaxBlocks * kLineWords;
constexpr int kSyncPart = kSyncJTag + kFlagCopies * kTagLines * kLineWords;
constexpr int kSyncWords = kSyncPart + 2 * kMaxBlocks * kTagLines * kLineWords;
constexpr int kTagWords64 = kTagLines * kLineWords / 2;   // 64-bit words per copy or slot

constexpr int kVacRows3 = 7;    // 3f table rows before the weights: 6 vacuum entries and e_k
constexpr int kBlock = 512;       // threads per block: the most a stepping launch uses (8 waves),
                                  // the size of their per-block LDS arrays
constexpr int kBlockSmall = 256;  // the other block size of the fixed-step kernels (4 waves)

// Arguments of the single-model stepping kernel (passed by value).
struct StepArgs {
  void* X;                 // state planes [nsc][plane] (double, or float for FP32 state)
  const double* tab;       // tables: 2f [bx|bz|G_0..G_{NS-1}] x NE; 3f [h_ee..h_mt (6)|e_k|G_s]
                           // x NE with e_k = 1/E_k; extended model: then cos, sin of every
                           // azimuthal bin
  unsigned int* sync;      // kSyncWords words (barrier words and the tagged reduction words)
  long long* step_ctl;     // [0] device step counter (read at launch start, advanced at the
                           // end); [1] target of a group of windowed launches
  long long plane;         // plane stride (elements)
  int NE, NU;
  int NP;                  // azimuthal bins (extended bulb model; 1 for the bulb model)
  int NS;                  // species rows: 2 (nu_e-, anti-nu_e-born) or 2 n_flavor (every
                           // flavour tracked; row s = anti * n_flavor + flavour of birth)
  long long nsteps, total_steps;  // requested steps (clamped to total_steps - start)
  double rs, h, R, lam0;
  int ne_power, renorm;
  double s1, s0, p2e1, p2e0;  // fixed-point scales 2^e1, 2^e0, 2^-e1, 2^-e0
  double v0[6];            // 3f: the vacuum Hamiltonian times E (entries of bin k = e_k v0)
  unsigned long long timeout_ticks;
  const unsigned* cancel;  // the model's cancel word (fine-grained host memory), or nullptr
  double* Jhist;           // nullptr, or [step][4][2*NC]: every stage's moments (adjoint tape)
  int use_window;          // 0: advance min(nsteps, total - step) steps; 1: the window below
  long long win_lo, win_hi;// windowed launch: only steps in [win_lo, win_hi), up to step_ctl[1]
  // adaptive step control (k_adaptive): second state buffer, tolerance^2, step limits, end
  void* X2;
  double tol2, hmax, hmin, r_end;
  long long max_attempts;
};
// step_ctl words of an adaptive run: [2] r, [3] h (double bits), [4] accepted, [5] rejected,
// [6] attempts, [7] 1 if the step control failed
constexpr int kCtlR = 2, kCtlH = 3, kCtlAcc = 4, kCtlRej = 5, kCtlAtt = 6, kCtlFail = 7;
// step_ctl words [kCtlMTag] and [kCtlMKind]: the step and the stepping-kernel variant whose
// stage-1 moments (those of the state at that step) the launch that ended there left in
// words [kCtlMom, kCtlMom + 32) as doubles, so that the next launch of the same variant
// skips its initial moment pass; kCtlMTag = -1: none (every change of the state outside a
// stepping launch sets it).
constexpr int kCtlMTag = 9, kCtlMKind = 10, kCtlMom = 16, kCtlWords = 48;

// One two-flavour model of a batch.
struct BatchModel {
  long long beam0;  // first beam of the model in the state planes
  long long row0;   // first global row; the model owns rows [row0, row0 + 2 NU)
  long long tab0;   // offset of its tables [bx|bz|G0|G1] x NE
  int NE, NU;
  double lam0;
  double s1, s0, p2e1, p2e0;
};

constexpr int kAccSets = 6;   // moment accumulator sets, rotated by barrier epoch
constexpr int kAccLimbs = 3;  // carry-save limbs of 42 bits per 128-bit sum

// Arguments of the batched two-flavour stepping kernel.
struct BatchArgs {
  double* X;
  long long plane;
  const double* tab;
  const BatchModel* models;
  int nmodels;
  const long long* wave_row0;   // [waves + 1]: each wavefront's contiguous row range
  long long total_rows;
  unsigned long long* acc;      // [kAccSets][nmodels][6][kAccLimbs]
  unsigned int* sync;
  long long* step_ctl;
  long long nsteps, total_steps;
  double rs, h, R;
  int ne_power, renorm;
  unsigned long long timeout_ticks;
  const unsigned* cancel;
};

// Arguments of the two-flavour reverse (adjoint) kernel.  Beam b belongs to thread
// b mod (grid threads); its adjoint state stays in registers for the whole launch, or, when
// the beams outnumber four per resident thread, in the workspace (spill).
struct AdjArgs {
  const double* tab;       // [bx|bz|G0|G1] x NE
  const double* dtab;      // [dG0/dL_e | dG1/dL_ebar | dG/dL_x | dbx/dtheta | dbz/dtheta] x NE
  const double* Jhist;     // [step][4][6] stage moments recorded by the forward pass
  const double* ck;        // [nseg][3][plane] state at the start of every segment
  double* tape;            // [ckpt][3][plane] states of the segment being reversed
  const double* cot;       // dL/dPee per beam, or nullptr: cot_const for every beam
  double cot_const;
  double* state_bar;       // nullptr, or [3][nb]: dL/d(state at the first step)
  double* spill;           // [9][plane]: the beams' adjoint registers (spill mode only)
  double* out;             // [8]: dL/d{L_e, L_ebar, L_x, theta_v, n0}
  unsigned int* sync;      // kSyncWords words (barrier words and the tagged reduction words)
  long long plane, nb;
  int NE, NU;
  long long n0, nsteps, ckpt, nseg;  // first step, steps, checkpoint period, segments
  double rs, h, R, lam0, s2gf;
  int ne_power, renorm;
  unsigned long long timeout_ticks;
  const unsigned* cancel;
};

}  // namespace nb
