// Synthetic environment stub for the environment-step loop of Alg. 1 (observe,
// act, step, store, then the UTD updates).  It stands in for the simulator and
// its batched renderer: a point mass driven by the action, a goal drawn per
// episode, and an integer renderer that draws the last three positions as discs
// into the frame stack.  One workgroup per environment: thread 0 advances the
// state (the workgroup owns it, so there are no races between environments),
// then all threads render.
#include "../common.h"
#include "philox.h"

namespace sq {

__device__ __forceinline__ int env_pix(float v, int side) {
  // (side / 8) v is exact (a power-of-two multiple for the sides used), so the sum
  // rounds once however the compiler contracts it
  const int q = (int)floorf((float)(side / 2) + (float)(side / 8) * v);
  return min(max(q, 0), side - 1);
}

// reset of environment e for episode ep: proprio in [-0.5, 0.5), goal in [-1.5, 1.5)
__device__ void env_reset(const EnvState& E, int e, int ep) {
  unsigned w[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const P4 r = philox10(P4{(unsigned)e, 5u, (unsigned)ep, (unsigned)q}, E.k0, E.k1);
    w[4 * q] = r.x;
    w[4 * q + 1] = r.y;
    w[4 * q + 2] = r.z;
    w[4 * q + 3] = r.w;
  }
  float* s = E.s + (long long)e * E.P;
  for (int j = 0; j < E.P; ++j) s[j] = 0.5f * (2.0f * uniform23(w[j]) - 1.0f);
  E.g[2 * e] = 1.5f * (2.0f * uniform23(w[12]) - 1.0f);
  E.g[2 * e + 1] = 1.5f * (2.0f * uniform23(w[13]) - 1.0f);
  E.t[e] = 0;
  E.ep[e] = ep;
  const int px = env_pix(s[0], E.W), py = env_pix(s[1], E.H);
  for (int k = 0; k < 3; ++k) {
    E.stack[6 * e + 2 * k] = px;
    E.stack[6 * e + 2 * k + 1] = py;
  }
}

// frame of environment e from its stack: slot k fills channels 3k..3k+2
__device__ void env_render(const EnvState& E, const int* stack, uint8_t* frame) {
  const int R2 = (E.H / 8) * (E.H / 8);
  const int n = E.H * E.W * E.C;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int c = i % E.C, px = (i / E.C) % E.W, py = i / (E.C * E.W);
    const int k = c / 3;
    const int dx = px - stack[2 * k], dy = py - stack[2 * k + 1];
    const int rgb = c - 3 * k;
    const unsigned v = dx * dx + dy * dy <= R2 ? (rgb == 0 ? 200u : rgb == 1 ? 120u : 40u)
                                               : (unsigned)((((px ^ py) * 5) + 11 * c) & 63);
    frame[i] = (uint8_t)v;
  }
}

__global__ __launch_bounds__(256) void k_env_reset(EnvState E, uint8_t* __restrict__ obs) {
  const int e = blockIdx.x;
  if (threadIdx.x == 0) env_reset(E, e, 0);
  __syncthreads();
  env_render(E, E.stack + 6 * e, obs + (long long)e * E.H * E.W * E.C);
}

// one step of environment e: writes the transition's next frame / proprio,
// reward and done, and the observation of the next step into obs_next
__global__ __launch_bounds__(256) void k_env_step(EnvState E, const float* __restrict__ action,
                                                  float* __restrict__ prop_t, uint8_t* __restrict__ next_obs,
                                                  float* __restrict__ next_prop, float* __restrict__ reward,
                                                  uint8_t* __restrict__ done, uint8_t* __restrict__ obs_next) {
  __shared__ int st[6];
  __shared__ int dn;
  const int e = blockIdx.x;
  const long long fb = (long long)E.H * E.W * E.C;
  if (threadIdx.x == 0) {
    float* s = E.s + (long long)e * E.P;
    const float* a = action + (long long)e * E.A;
    for (int j = 0; j < E.P; ++j) {
      prop_t[(long long)e * E.P + j] = s[j];
      s[j] = fminf(fmaxf(s[j] + a[j % E.A] * 0.125f, -2.0f), 2.0f);
      next_prop[(long long)e * E.P + j] = s[j];
    }
    const float d0 = s[0] - E.g[2 * e], d1 = s[1] - E.g[2 * e + 1];
    reward[e] = -(d0 * d0 + d1 * d1);
    const int t = E.t[e] + 1;
    const int d = t == E.T;
    done[e] = (uint8_t)d;
    E.t[e] = t;
    int* sk = E.stack + 6 * e;
    st[0] = env_pix(s[0], E.W);
    st[1] = env_pix(s[1], E.H);
    st[2] = sk[0];
    st[3] = sk[1];
    st[4] = sk[2];
    st[5] = sk[3];
    for (int i = 0; i < 6; ++i) sk[i] = st[i];
    if (d) env_reset(E, e, E.ep[e] + 1);
    dn = d;
  }
  __syncthreads();
  env_render(E, st, next_obs + e * fb);
  if (dn) env_render(E, E.stack + 6 * e, obs_next + e * fb);
  else env_render(E, st, obs_next + e * fb);
}

int env_reset_all(const EnvState& E, uint8_t* obs, hipStream_t st) {
  k_env_reset<<<E.n, 256, 0, st>>>(E, obs);
  return launch_status("env_reset");
}

int env_step(const EnvState& E, const float* action, float* prop_t, uint8_t* next_obs, float* next_prop,
             float* reward, uint8_t* done, uint8_t* obs_next, hipStream_t st) {
  k_env_step<<<E.n, 256, 0, st>>>(E, action, prop_t, next_obs, next_prop, reward, done, obs_next);
  return launch_status("env_step");
}

}  // namespace sq
