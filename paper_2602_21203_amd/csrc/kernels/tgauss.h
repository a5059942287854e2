// The tanh-Gaussian policy head (Sec. III, Eq. (3)): head = [mu | u_s],
// log sigma = lo + (hi - lo) (tanh u_s + 1) / 2, u = mu + sigma eps, a = tanh u,
// log pi = sum_d [N(eps; 0, 1) log-density - log sigma - log(1 - tanh^2 u)], the
// last term written as 2 (log 2 - u - softplus(-2u)).  save = (tanh u_s, sigma, a)
// for the backward.  Shared by the standalone kernel and the GEMM epilogue that
// produces the head, so both give the same arithmetic; log pi sums the dimension
// terms in d order in both.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace sq {

__device__ __forceinline__ float tg_softplus(float x) { return x > 0.f ? x + log1pf(expf(-x)) : log1pf(expf(x)); }

// dimension d of one row: writes action[d] and the row's save entries of d; returns
// the log-density term of d
__device__ __forceinline__ float tanh_gauss_dim(float mu, float us, float e, int A, int d, float lo, float hi,
                                                float* __restrict__ action, float* __restrict__ save) {
  const float half_log_2pi = 0.91893853320467274f;
  const float log2 = 0.69314718055994531f;
  const float tus = tanhf(us);
  const float ls = lo + 0.5f * (hi - lo) * (tus + 1.f);
  const float sd = expf(ls);
  const float u = mu + sd * e;
  const float a = tanhf(u);
  action[d] = a;
  save[d] = tus;
  save[A + d] = sd;
  save[2 * A + d] = a;
  return -0.5f * e * e - ls - half_log_2pi - 2.f * (log2 - u - tg_softplus(-2.f * u));
}

}  // namespace sq
