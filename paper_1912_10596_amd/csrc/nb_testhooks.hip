// nb_testhooks.hip -- libnubulb_testhooks.so: the stepper's arithmetic primitives (the
// two-flavour sin/cos and rotation, the three-flavour exponential, hardware sqrt and
// division), one element per thread, so that tests can hold each to its definition.  Built
// from the same device headers as the stepping kernels; not part of the stepper's ABI.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/nubulb_testhooks.h"
#include "nb_device.h"

namespace nb {
__global__ void k_test_sincos(const double* x, long long n, double* s, double* c) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a, b;
  sincos_nb(x[i], a, b);
  s[i] = a;
  c[i] = b;
}
__global__ void k_test_sqrt_div(const double* a, const double* b, long long n, double* sq, double* dv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  sq[i] = sqrt(a[i]);
  dv[i] = a[i] / b[i];
}
__global__ void k_test_exp3(const double* k9, const double* psi6, long long n, double* out6) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* k = k9 + 9 * i;
  const Herm3 K{k[0], k[1], k[2], mk(k[3], k[4]), mk(k[5], k[6]), mk(k[7], k[8])};
  const double* p = psi6 + 6 * i;
  cplx ps[3] = {mk(p[0], p[1]), mk(p[2], p[3]), mk(p[4], p[5])};
  exp3_apply(K, ps);
  double* o = out6 + 6 * i;
  for (int c = 0; c < 3; ++c) {
    o[2 * c] = ps[c].re;
    o[2 * c + 1] = ps[c].im;
  }
}
__global__ void k_test_rotate(const double* x3, const double* p3, long long n, double* out3) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double P0 = p3[3 * i], P1 = p3[3 * i + 1], P2 = p3[3 * i + 2];
  rotate2(x3[3 * i], x3[3 * i + 1], x3[3 * i + 2], P0, P1, P2);
  out3[3 * i] = P0;
  out3[3 * i + 1] = P1;
  out3[3 * i + 2] = P2;
}

}  // namespace nb

using namespace nb;

static thread_local std::string g_err;
static int fail(int code, const char* fmt, ...) {
  char buf[256];
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
    if (e_ != hipSuccess) return fail(NB_TEST_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* nb_test_last_error(void) { return g_err.c_str(); }

static int launch_1d(const void* fn, long long n, void** args, hipStream_t s) {
  const int bs = 256;
  const long long nblk = (n + bs - 1) / bs;
  if (nblk <= 0) return NB_TEST_OK;
  NB_HIP(hipLaunchKernel(fn, dim3((unsigned)nblk), dim3(bs), args, 0, s));
  return NB_TEST_OK;
}

extern "C" int nb_test_sincos(const double* x, int64_t n, double* s, double* c, void* stream) {
  if (n < 0 || (n > 0 && (!x || !s || !c))) return fail(NB_TEST_EINVAL, "bad arguments");
  long long nn = n;
  void* args[] = {&x, &nn, &s, &c};
  int rc = launch_1d((const void*)&k_test_sincos, n, args, (hipStream_t)stream);
  if (rc) return rc;
  NB_HIP(hipStreamSynchronize((hipStream_t)stream));
  return NB_TEST_OK;
}
extern "C" int nb_test_sqrt_div(const double* a, const double* b, int64_t n, double* sq, double* dv,
                                void* stream) {
  if (n < 0 || (n > 0 && (!a || !b || !sq || !dv))) return fail(NB_TEST_EINVAL, "bad arguments");
  long long nn = n;
  void* args[] = {&a, &b, &nn, &sq, &dv};
  int rc = launch_1d((const void*)&k_test_sqrt_div, n, args, (hipStream_t)stream);
  if (rc) return rc;
  NB_HIP(hipStreamSynchronize((hipStream_t)stream));
  return NB_TEST_OK;
}
extern "C" int nb_test_exp3(const double* k9, const double* psi6, int64_t n, double* out6, void* stream) {
  if (n < 0 || (n > 0 && (!k9 || !psi6 || !out6))) return fail(NB_TEST_EINVAL, "bad arguments");
  long long nn = n;
  void* args[] = {&k9, &psi6, &nn, &out6};
  int rc = launch_1d((const void*)&k_test_exp3, n, args, (hipStream_t)stream);
  if (rc) return rc;
  NB_HIP(hipStreamSynchronize((hipStream_t)stream));
  return NB_TEST_OK;
}
extern "C" int nb_test_rotate(const double* x3, const double* p3, int64_t n, double* out3, void* stream) {
  if (n < 0 || (n > 0 && (!x3 || !p3 || !out3))) return fail(NB_TEST_EINVAL, "bad arguments");
  long long nn = n;
  void* args[] = {&x3, &p3, &nn, &out3};
  int rc = launch_1d((const void*)&k_test_rotate, n, args, (hipStream_t)stream);
  if (rc) return rc;
  NB_HIP(hipStreamSynchronize((hipStream_t)stream));
  return NB_TEST_OK;
}
