/*
 * nubulb_testhooks.h -- C-ABI of libnubulb_testhooks.so, a separate library that exposes
 * the arithmetic primitives of the stepper one element per thread, built from the same
 * device code as the stepping kernels, so that tests can check each against its
 * definition.  Not part of the stepper's ABI (include/nubulb.h); nothing in libnubulb.so
 * depends on it.
 *
 * Every entry point: dev_* are device arrays of n elements (n * 9 for k9, n * 6 for psi6,
 * n * 3 for x3 and p3), owned by the caller; the work is enqueued on `stream` (a
 * hipStream_t, may be NULL) and the call returns after the stream has drained.  Returns
 * NB_TEST_OK, or NB_TEST_EINVAL (negative n or a NULL array with n > 0) / NB_TEST_EHIP (a
 * HIP call failed); nb_test_last_error() then holds a message for the calling thread.
 */
#ifndef NUBULB_TESTHOOKS_H
#define NUBULB_TESTHOOKS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { NB_TEST_OK = 0, NB_TEST_EINVAL = -1, NB_TEST_EHIP = -4 };

/* sin and cos of the two-flavour rotation angle (the stepper's own polynomial evaluation). */
int nb_test_sincos(const double *dev_x, int64_t n, double *dev_s, double *dev_c, void *stream);
/* Hardware FP64 square root and division, element by element (IEEE correctly rounded). */
int nb_test_sqrt_div(const double *dev_a, const double *dev_b, int64_t n, double *dev_sqrt,
                     double *dev_div, void *stream);
/* exp(-i K) psi, up to a global phase, for a Hermitian 3x3 generator K given as (K_ee,
 * K_mm, K_tt, Re/Im K_em, Re/Im K_et, Re/Im K_mt) and psi as Re/Im of (psi_e, psi_mu,
 * psi_tau) (the one-step propagator of Eq. U, three flavours). */
int nb_test_exp3(const double *dev_k9, const double *dev_psi6, int64_t n, double *dev_out6,
                 void *stream);
/* Rotation of the Bloch vector p3 about the axis x3 by the angle |x3| (two-flavour Eq. U). */
int nb_test_rotate(const double *dev_x3, const double *dev_p3, int64_t n, double *dev_out3,
                   void *stream);
const char *nb_test_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
