// nyx_mlp.hip -- training and packing kernels of the learned Riemann flux
// (the network is described in nyx_mlp_dev.h).  Training runs in FP32 on the
// vector units: one thread per sample computes its forward pass, loss and
// backpropagated gradient; per-weight gradients are summed over each
// wavefront with shuffles and accumulated with one atomic per wavefront.  The
// optimiser is Adam.  Packing converts the FP32 master weights into the BF16
// MFMA fragments the inference path reads.
#include <hip/hip_runtime.h>

#include "nyx_internal.h"
#include "nyx_mlp_dev.h"

namespace nyx {

// normalisation of a harvested record (15 floats: left state, right state,
// p*, u*, rho*_L, rho*_R, rho_g); inputs x[10] and targets y[5]
__device__ __forceinline__ void record_xy(double gamma, const float* r, float* x, float* y) {
  double qL[5], qR[5];
  for (int k = 0; k < 5; ++k) {
    qL[k] = (double)r[k];
    qR[k] = (double)r[5 + k];
  }
  double rbar, cbar, ubar;
  mlp_inputs(gamma, qL, qR, x, &rbar, &cbar, &ubar);
  if (y) {
    const double pbar = rbar * cbar * cbar;
    y[0] = (float)log((double)r[10] / pbar);
    y[1] = (float)(((double)r[11] - ubar) / cbar);
    y[2] = (float)log((double)r[12] / rbar);
    y[3] = (float)log((double)r[13] / rbar);
    y[4] = (float)log((double)r[14] / rbar);
  }
}

__device__ __forceinline__ float wave_sumf(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// splitmix64 of (seed, i) -> uniform in [0, 1)
__device__ __forceinline__ double uniform01(unsigned long long seed, unsigned long long i) {
  unsigned long long z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Glorot-uniform weights, zero biases
__global__ void k_mlp_init(float* P, unsigned long long seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpNParam) return;
  int nin = 0, nout = 0;
  bool bias = false;
  if (i < kOffB1) { nin = kMlpIn; nout = kMlpHid; }
  else if (i < kOffW2) bias = true;
  else if (i < kOffB2) { nin = kMlpHid; nout = kMlpHid; }
  else if (i < kOffW3) bias = true;
  else if (i < kOffB3) { nin = kMlpHid; nout = kMlpHid; }
  else if (i < kOffW4) bias = true;
  else if (i < kOffB4) { nin = kMlpHid; nout = kMlpOut; }
  else bias = true;
  if (bias) {
    P[i] = 0.0f;
    return;
  }
  const double lim = sqrt(6.0 / (double)(nin + nout));
  P[i] = (float)((2.0 * uniform01(seed, (unsigned long long)i) - 1.0) * lim);
}

// dense layer out[o] = b[o] + sum_i W[o][i] in[i] (weights read uniformly)
template <int NIN, int NOUT, bool RELU>
__device__ __forceinline__ void dense_f(const float* __restrict__ W, const float* __restrict__ b,
                                        const float* in, float* out) {
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    float acc = b[o];
#pragma unroll
    for (int i = 0; i < NIN; ++i) acc += W[o * NIN + i] * in[i];
    out[o] = RELU ? (acc > 0.0f ? acc : 0.0f) : acc;
  }
}

// accumulate grad W[o][i] += sum over the wave of d[o] in[i], grad b[o] += sum d[o]
template <int NIN, int NOUT>
__device__ __forceinline__ void accum_grad(float* __restrict__ gW, float* __restrict__ gb,
                                           const float* d, const float* in, bool lead) {
#pragma unroll 1
  for (int o = 0; o < NOUT; ++o) {
    const float s = wave_sumf(d[o]);
    if (lead && s != 0.0f) atomicAdd(gb + o, s);
#pragma unroll 4
    for (int i = 0; i < NIN; ++i) {
      const float v = wave_sumf(d[o] * in[i]);
      if (lead && v != 0.0f) atomicAdd(gW + o * NIN + i, v);
    }
  }
}

// back through a dense layer: dprev[i] = mask(h_prev[i]) * sum_o W[o][i] d[o]
template <int NIN, int NOUT>
__device__ __forceinline__ void back_f(const float* __restrict__ W, const float* d,
                                       const float* hprev, float* dprev) {
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) acc += W[o * NIN + i] * d[o];
    dprev[i] = hprev[i] > 0.0f ? acc : 0.0f;
  }
}

// loss and gradient of a batch chunk; grad and loss are accumulated (the
// caller zeroes them); `inv_n` = 1 / (samples in the whole batch)
__global__ __launch_bounds__(64) void k_mlp_loss_grad(const float* __restrict__ P,
                                                      const float* __restrict__ rec, long long n,
                                                      double gamma, float inv_n,
                                                      float* __restrict__ grad, float* loss) {
  const long long s = (long long)blockIdx.x * 64 + threadIdx.x;
  bool valid = s < n;
  const bool lead = (threadIdx.x & 63) == 0;
  float x[kMlpIn], y[kMlpOut];
  if (valid) {
    record_xy(gamma, rec + 15 * s, x, y);
    // only samples inside the training domain enter the loss
    for (int k = 0; k < kMlpIn; ++k) valid = valid && fabsf(x[k]) <= kMlpDomain;
    for (int k = 0; k < kMlpOut; ++k) valid = valid && fabsf(y[k]) <= kMlpDomain;
  }
  if (!valid) {
    for (int k = 0; k < kMlpIn; ++k) x[k] = 0.0f;
    for (int k = 0; k < kMlpOut; ++k) y[k] = 0.0f;
  }
  float h1[kMlpHid], h2[kMlpHid], h3[kMlpHid], yh[kMlpOut];
  dense_f<kMlpIn, kMlpHid, true>(P + kOffW1, P + kOffB1, x, h1);
  dense_f<kMlpHid, kMlpHid, true>(P + kOffW2, P + kOffB2, h1, h2);
  dense_f<kMlpHid, kMlpHid, true>(P + kOffW3, P + kOffB3, h2, h3);
  dense_f<kMlpHid, kMlpOut, false>(P + kOffW4, P + kOffB4, h3, yh);
  float d4[kMlpOut], l2 = 0.0f;
  for (int o = 0; o < kMlpOut; ++o) {
    const float e = valid ? yh[o] - y[o] : 0.0f;
    l2 += e * e;
    d4[o] = 2.0f * e * inv_n;
  }
  const float ls = wave_sumf(l2);
  if (lead) atomicAdd(loss, ls * inv_n);
  accum_grad<kMlpHid, kMlpOut>(grad + kOffW4, grad + kOffB4, d4, h3, lead);
  float d3[kMlpHid];
  back_f<kMlpHid, kMlpOut>(P + kOffW4, d4, h3, d3);
  accum_grad<kMlpHid, kMlpHid>(grad + kOffW3, grad + kOffB3, d3, h2, lead);
  float d2[kMlpHid];
  back_f<kMlpHid, kMlpHid>(P + kOffW3, d3, h2, d2);
  accum_grad<kMlpHid, kMlpHid>(grad + kOffW2, grad + kOffB2, d2, h1, lead);
  float d1[kMlpHid];
  back_f<kMlpHid, kMlpHid>(P + kOffW2, d2, h1, d1);
  accum_grad<kMlpIn, kMlpHid>(grad + kOffW1, grad + kOffB1, d1, x, lead);
}

__global__ void k_mlp_adam(float* P, float* m, float* v, const float* g, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpNParam) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP32 master weights -> BF16 MFMA fragments + FP32 (padded) biases
__global__ void k_mlp_pack(const float* P, unsigned char* packed) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kMlpFrags * 64 * 8) {
    const int f = t / 512, l = (t / 8) % 64, e = t % 8;
    int layer, m, s;
    if (f < 2) { layer = 0; m = f; s = 0; }
    else if (f < 10) { layer = 1; m = (f - 2) / 4; s = (f - 2) % 4; }
    else if (f < 18) { layer = 2; m = (f - 10) / 4; s = (f - 10) % 4; }
    else { layer = 3; m = 0; s = f - 18; }
    const int row = 32 * m + (l & 31), k = 16 * s + 8 * (l >> 5) + e;
    const int nin = layer == 0 ? kMlpIn : kMlpHid;
    const int nout = layer == 3 ? kMlpOut : kMlpHid;
    const int woff = layer == 0 ? kOffW1 : (layer == 1 ? kOffW2 : (layer == 2 ? kOffW3 : kOffW4));
    const float w = (row < nout && k < nin) ? P[woff + row * nin + k] : 0.0f;
    ((__bf16*)packed)[t] = (__bf16)w;
  } else if (t < kMlpFrags * 64 * 8 + 224) {
    const int j = t - kMlpFrags * 64 * 8;
    float b;
    if (j < 64) b = P[kOffB1 + j];
    else if (j < 128) b = P[kOffB2 + j - 64];
    else if (j < 192) b = P[kOffB3 + j - 128];
    else b = (j - 192) < kMlpOut ? P[kOffB4 + j - 192] : 0.0f;
    ((float*)(packed + kMlpBiasOff))[j] = b;
  }
}

// inference on harvested records (BF16 MFMA path): out[n][5]
__global__ __launch_bounds__(256) void k_mlp_predict(const void* packed, const float* rec,
                                                      long long n, double gamma, float* out) {
  __shared__ __bf16 lds[4 * kMlpWaveLds];
  const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
  float x[kMlpIn];
  if (s < n) {
    record_xy(gamma, rec + 15 * s, x, nullptr);
  } else {
    for (int k = 0; k < kMlpIn; ++k) x[k] = 1.0f;
  }
  float y[kMlpOut];
  mlp_wave_forward(packed, x, lds + (threadIdx.x >> 6) * kMlpWaveLds, y);
  if (s < n)
    for (int k = 0; k < kMlpOut; ++k) out[5 * s + k] = y[k];
}

// ---- launchers ----
hipError_t launch_mlp_init(float* P, unsigned long long seed, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_init, dim3((kMlpNParam + 255) / 256), dim3(256), 0, st, P, seed);
  return hipGetLastError();
}
hipError_t launch_mlp_loss_grad(const float* P, const float* rec, long long n, double gamma,
                                float inv_n, float* grad, float* loss, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_loss_grad, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, P, rec, n,
                     gamma, inv_n, grad, loss);
  return hipGetLastError();
}
hipError_t launch_mlp_adam(float* P, float* m, float* v, const float* g, int t, float lr, float b1,
                           float b2, float eps, hipStream_t st) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpNParam + 255) / 256), dim3(256), 0, st, P, m, v, g, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t launch_mlp_pack(const float* P, void* packed, hipStream_t st) {
  const int n = kMlpFrags * 64 * 8 + 224;
  hipLaunchKernelGGL(k_mlp_pack, dim3((n + 255) / 256), dim3(256), 0, st, P,
                     (unsigned char*)packed);
  return hipGetLastError();
}
hipError_t launch_mlp_predict(const void* packed, const float* rec, long long n, double gamma,
                              float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, packed,
                     rec, n, gamma, out);
  return hipGetLastError();
}

}  // namespace nyx
