// nyx_mlp_dev.h -- device side of the learned Riemann flux: input
// normalisation and the wave-wide BF16 MFMA forward pass of the network
// 10 -> 64 -> 64 -> 64 -> 5 (ReLU hidden layers, FP32 accumulation).
//
// A face is described by its rotated left/right states (rho, u_n, u_t1,
// u_t2, p).  With c_K = sqrt(gamma p_K/rho_K), rbar, cbar, ubar the means of
// the two densities, sound speeds and normal velocities and Pbar = rbar cbar^2,
// the network input is
//   (rho_L/rbar, (u_L-ubar)/cbar, v_L/cbar, w_L/cbar, p_L/Pbar, same for R)
// and its outputs approximate
//   (ln(p*/Pbar), (u*-ubar)/cbar, ln(rho*_L/rbar), ln(rho*_R/rbar), ln(rho_g/rbar))
// of the two-shock solution (p*, u* star pressure and velocity, rho*_K star
// densities, rho_g density of the Godunov state).
//
// Forward pass on MFMA: one wavefront evaluates 64 faces together.  Faces are
// the N dimension of v_mfma_f32_32x32x16_bf16 (D[32x32] += A[32x16] B[16x32]):
// A holds weight fragments (rows = output units), B the activations of 32
// faces, read from a per-wave LDS tile [face][feature] in BF16.  Biases
// initialise the accumulators.  Operand layouts (checked on gfx950):
//   A: lane l, element e = A[l%32][8(l/32)+e];  B: lane l, e = B[8(l/32)+e][l%32]
//   D: lane l, element v = D[8(v/4)+4(l/32)+v%4][l%32].
#pragma once
#include <hip/hip_runtime.h>

namespace nyx {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMlpIn = 10, kMlpHid = 64, kMlpOut = 5;
// Training domain: a face's normalised inputs and targets must be finite and
// at most this large in magnitude (floored pressures or near-vacuum faces
// normalise to huge values; they are left out of training and, in a step,
// fall back to the two-shock solver).
constexpr float kMlpDomain = 64.0f;
constexpr int kMlpNParam = kMlpHid * kMlpIn + kMlpHid + 2 * (kMlpHid * kMlpHid + kMlpHid) +
                           kMlpOut * kMlpHid + kMlpOut;  // 9349
// offsets in the flat FP32 parameter vector: W[o][i] row-major, then b
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpHid * kMlpIn, kOffW2 = kOffB1 + kMlpHid,
              kOffB2 = kOffW2 + kMlpHid * kMlpHid, kOffW3 = kOffB2 + kMlpHid,
              kOffB3 = kOffW3 + kMlpHid * kMlpHid, kOffW4 = kOffB3 + kMlpHid,
              kOffB4 = kOffW4 + kMlpOut * kMlpHid;
// packed inference weights: 22 fragments of 64 lanes x 8 bf16, then biases
// (FP32: 64 + 64 + 64 + 32 with the last layer padded to 32 rows)
constexpr int kMlpFrags = 22;
constexpr int kMlpBiasOff = kMlpFrags * 64 * 16;           // bytes
constexpr int kMlpPackedBytes = kMlpBiasOff + 224 * 4 + 128;  // 23552
constexpr int kMlpRow = 72;                                // bf16 per LDS row (64 + 8 pad)
constexpr int kMlpWaveLds = 64 * kMlpRow;                  // bf16 per wavefront

// first fragment of each layer and its K steps (fragment = fbase + Mt*nK + s)
__host__ __device__ constexpr int mlp_fbase(int layer) {
  return layer == 0 ? 0 : (layer == 1 ? 2 : (layer == 2 ? 10 : 18));
}
__host__ __device__ constexpr int mlp_nk(int layer) { return layer == 0 ? 1 : 4; }

// FP64 reciprocal and reciprocal square root: hardware estimate (relative
// error below 2^-24) and one Newton step, about 2^-47; positive arguments.
__device__ __forceinline__ double mlp_rcp(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double mlp_rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-(x * y), y, 1.0), y);
}

// Normalised inputs of one face (float) from rotated states in double.  The
// inputs are rounded to float (and to BF16 in the network), so the scalings
// are products with refined reciprocals instead of divisions.  A non-positive
// or non-finite state gives a non-finite or huge input, which the caller's
// domain test sends to the plain solver.
__device__ __forceinline__ void mlp_inputs(double gamma, const double* qL, const double* qR,
                                           float* x, double* rbar_o, double* cbar_o,
                                           double* ubar_o) {
  const double sl = gamma * qL[4] * mlp_rcp(qL[0]);
  const double sr = gamma * qR[4] * mlp_rcp(qR[0]);
  const double cl = sl * mlp_rsq(sl);
  const double cr = sr * mlp_rsq(sr);
  const double rbar = 0.5 * (qL[0] + qR[0]);
  const double cbar = 0.5 * (cl + cr);
  const double ubar = 0.5 * (qL[1] + qR[1]);
  const double pbar = rbar * cbar * cbar;
  const double ir = mlp_rcp(rbar), ic = mlp_rcp(cbar), ip = mlp_rcp(pbar);
  x[0] = (float)(qL[0] * ir);
  x[1] = (float)((qL[1] - ubar) * ic);
  x[2] = (float)(qL[2] * ic);
  x[3] = (float)(qL[3] * ic);
  x[4] = (float)(qL[4] * ip);
  x[5] = (float)(qR[0] * ir);
  x[6] = (float)((qR[1] - ubar) * ic);
  x[7] = (float)(qR[2] * ic);
  x[8] = (float)(qR[3] * ic);
  x[9] = (float)(qR[4] * ip);
  *rbar_o = rbar;
  *cbar_o = cbar;
  *ubar_o = ubar;
}

// Wave-wide forward pass.  Every lane of the wavefront must call it (inactive
// faces pass any finite inputs).  x: this lane's 10 inputs; lds: this wave's
// kMlpWaveLds bf16 scratch.  Returns the 5 outputs of this lane's face.
__device__ __forceinline__ void mlp_wave_forward(const void* packed, const float* x,
                                                 __bf16* lds, float* y) {
  const int l = threadIdx.x & 63;
  const int hi = l >> 5, col = l & 31;
  const bf16x8* F = (const bf16x8*)packed;
  const float* Bv = (const float*)((const char*)packed + kMlpBiasOff);
  __bf16* row = lds + l * kMlpRow;
  for (int k = 0; k < 16; ++k) row[k] = (__bf16)(k < kMlpIn ? x[k] : 0.0f);
  __builtin_amdgcn_wave_barrier();
  // three hidden layers
  for (int layer = 0; layer < 3; ++layer) {
    const int nK = mlp_nk(layer), fb = mlp_fbase(layer);
    const float* bias = Bv + 64 * layer;
    f32x16 acc[2][2];
    for (int m = 0; m < 2; ++m)
      for (int v = 0; v < 16; ++v) {
        const float bv = bias[32 * m + 8 * (v >> 2) + 4 * hi + (v & 3)];
        acc[0][m][v] = bv;
        acc[1][m][v] = bv;
      }
    for (int s = 0; s < nK; ++s) {
      bf16x8 b[2];
      for (int t = 0; t < 2; ++t)
        b[t] = *(const bf16x8*)(lds + (32 * t + col) * kMlpRow + 16 * s + 8 * hi);
      for (int m = 0; m < 2; ++m) {
        const bf16x8 a = F[(fb + m * nK + s) * 64 + l];
        for (int t = 0; t < 2; ++t)
          acc[t][m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[t], acc[t][m], 0, 0, 0);
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (int t = 0; t < 2; ++t)
      for (int m = 0; m < 2; ++m)
        for (int j = 0; j < 4; ++j) {
          bf16x4 w;
          for (int q = 0; q < 4; ++q) {
            const float z = acc[t][m][4 * j + q];
            // ReLU on the bits: a negative float is a negative integer
            w[q] = (__bf16)__int_as_float(max(__float_as_int(z), 0));
          }
          *(bf16x4*)(lds + (32 * t + col) * kMlpRow + 32 * m + 8 * j + 4 * hi) = w;
        }
    __builtin_amdgcn_wave_barrier();
  }
  // output layer: one 32-row tile (rows 0..4 used)
  f32x16 out[2];
  for (int v = 0; v < 16; ++v) {
    const float bv = Bv[192 + 8 * (v >> 2) + 4 * hi + (v & 3)];
    out[0][v] = bv;
    out[1][v] = bv;
  }
  for (int s = 0; s < 4; ++s) {
    const bf16x8 a = F[(mlp_fbase(3) + s) * 64 + l];
    for (int t = 0; t < 2; ++t) {
      const bf16x8 b = *(const bf16x8*)(lds + (32 * t + col) * kMlpRow + 16 * s + 8 * hi);
      out[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, out[t], 0, 0, 0);
    }
  }
  // face i < 32: outputs 0..3 in lane i (tile 0, v = 0..3), output 4 in lane
  // i + 32 (tile 0, v = 0); face i >= 32: outputs 0..3 in lane i - 32 (tile 1),
  // output 4 in lane i (tile 1, v = 0)
  const int src = hi ? l - 32 : l;
  float o0 = __shfl(out[1][0], src, 64), o1 = __shfl(out[1][1], src, 64);
  float o2 = __shfl(out[1][2], src, 64), o3 = __shfl(out[1][3], src, 64);
  const float o4 = __shfl(out[0][0], (l + 32) & 63, 64);
  if (!hi) {
    o0 = out[0][0];
    o1 = out[0][1];
    o2 = out[0][2];
    o3 = out[0][3];
  }
  y[0] = o0;
  y[1] = o1;
  y[2] = o2;
  y[3] = o3;
  y[4] = hi ? out[1][0] : o4;
}

}  // namespace nyx
