// Learned scheduler: a 3 -> 64 -> 64 -> 1 network (ReLU, logit output) that
// scores pending vertices; a round then takes the top ceil(q n) vertices by
// priority x sigmoid(score) instead of by priority alone. The network is
// trained on the device on traces of plain exact top-k runs. Forward and
// backward products run on BF16 MFMA (v_mfma_f32_16x16x16_bf16) with FP32
// accumulation; master weights and Adam moments are FP32.
//
// Per wavefront, a tile of 16 samples is pushed through transposed products
// Z^T = W X^T: the 16x16 FP32 output tile of one layer, held four values per
// lane, is exactly the B operand of the next layer once rounded to BF16, so the
// forward pass needs no data movement between layers. Weight gradients need
// the transposed operands and go through a small per-wave LDS buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "daic_device.h"
#include "daic_internal.h"
#include "daic_kernels.h"
#include "daic_problem.h"

namespace daic {

constexpr int kIn = 3, kH = 64;
constexpr int kNParams = kH * kIn + kH + kH * kH + kH + kH + 1;  // 4481
// offsets of the FP32 parameter vector
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH;

typedef short bf16x4 __attribute__((__vector_size__(4 * sizeof(short))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __host__ inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// BF16 copies of the weights in the layouts the tiles read.
struct MlpDev {
  const uint16_t* W1b;  // [64][4]  (input features 0..2, column 3 zero)
  const uint16_t* W2b;  // [64][64] (out, in)
  const uint16_t* W3b;  // [64]
  const float* b1;      // [64]
  const float* b2;      // [64]
  const float* b3;      // [1]
};

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Forward of one 16-sample tile. Lane l holds sample s = l % 16 and, for the
// per-layer outputs, hidden units 16 t + 4 (l / 16) + i (i = 0..3) of tile t.
//   x: this lane's sample features (used by lanes 0..15 only).
// Outputs z1/z2 (pre-activations, FP32) and the logit of sample l (lanes 0..15).
struct TileAct {
  f32x4 z1[4], z2[4];
  bf16x4 h1[4], h2[4];
  float logit;
};

__device__ __forceinline__ void tile_forward(const MlpDev& m, float x0, float x1, float x2, TileAct& t) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t q = lane >> 4, r = lane & 15;
  // B operand of layer 1: X^T, k = feature 4q + i, n = sample r
  bf16x4 bx;
  if (q == 0) {
    bx[0] = (short)f2bf(x0);
    bx[1] = (short)f2bf(x1);
    bx[2] = (short)f2bf(x2);
    bx[3] = 0;
  } else {
    bx[0] = bx[1] = bx[2] = bx[3] = 0;
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    bf16x4 a;  // A = W1 rows 16 mt + r, columns 4q + i
    if (q == 0) {
      const uint16_t* w = m.W1b + (16 * mt + r) * 4;
      a[0] = (short)w[0];
      a[1] = (short)w[1];
      a[2] = (short)w[2];
      a[3] = (short)w[3];
    } else {
      a[0] = a[1] = a[2] = a[3] = 0;
    }
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    z = mfma16(a, bx, z);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z[i] += m.b1[16 * mt + 4 * q + i];
      t.h1[mt][i] = (short)f2bf(z[i] > 0.f ? z[i] : 0.f);
    }
    t.z1[mt] = z;
  }
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      const uint16_t* w = m.W2b + (16 * ot + r) * kH + 16 * kt + 4 * q;
      bf16x4 a;
      a[0] = (short)w[0];
      a[1] = (short)w[1];
      a[2] = (short)w[2];
      a[3] = (short)w[3];
      z = mfma16(a, t.h1[kt], z);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z[i] += m.b2[16 * ot + 4 * q + i];
      t.h2[ot][i] = (short)f2bf(z[i] > 0.f ? z[i] : 0.f);
    }
    t.z2[ot] = z;
  }
  f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) {
    bf16x4 a;  // A = W3 padded to 16 rows: row 0 real
    if (r == 0) {
      const uint16_t* w = m.W3b + 16 * kt + 4 * q;
      a[0] = (short)w[0];
      a[1] = (short)w[1];
      a[2] = (short)w[2];
      a[3] = (short)w[3];
    } else {
      a[0] = a[1] = a[2] = a[3] = 0;
    }
    z = mfma16(a, t.h2[kt], z);
  }
  // row 0 of the output tile: lanes 0..15, element 0
  t.logit = z[0] + m.b3[0];
}

__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev m, const float* x, uint64_t N, float* logits) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = (uint64_t)gridDim.x * 4;
  for (uint64_t tile = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile * 16 < N; tile += waves) {
    const uint64_t s = tile * 16 + (lane & 15);
    float x0 = 0.f, x1 = 0.f, x2 = 0.f;
    if (s < N) {
      x0 = x[s * 3];
      x1 = x[s * 3 + 1];
      x2 = x[s * 3 + 2];
    }
    TileAct t;
    tile_forward(m, x0, x1, x2, t);
    if (lane < 16 && s < N) logits[s] = t.logit;
  }
}

// Gradient of the mean BCE-with-logits loss over N samples, accumulated per
// wave and written as per-wave partials [waves][kNParams] (plus the loss sum).
// LDS per wave: dZ^T and activations^T as BF16 [64 rows][16 samples].
__global__ __launch_bounds__(256) void k_mlp_grad(MlpDev m, const float* x, const float* y, uint64_t N,
                                                  double inv_total, float* part, double* part_loss) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t q = lane >> 4, r = lane & 15;
  __shared__ uint16_t s_dz[4][kH][16];
  __shared__ uint16_t s_act[4][kH][16];
  // accumulators
  f32x4 gW2[4][4];
  f32x4 gW1[4];
  float gb1[4][4], gb2[4][4], gW3[4][4];
  float gb3 = 0.f;
  double loss = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      gb1[a][b] = gb2[a][b] = gW3[a][b] = 0.f;
    }
  }
  const uint64_t waves = (uint64_t)gridDim.x * 4;
  for (uint64_t tile = (uint64_t)blockIdx.x * 4 + wave; tile * 16 < N; tile += waves) {
    const uint64_t s = tile * 16 + r;
    const bool valid = s < N;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, yy = 0.f;
    if (valid) {
      x0 = x[s * 3];
      x1 = x[s * 3 + 1];
      x2 = x[s * 3 + 2];
      yy = y[s];
    }
    TileAct t;
    tile_forward(m, x0, x1, x2, t);
    // dL/dlogit for sample r (every lane of the column computes the same)
    const float zl = __shfl(t.logit, (int)r, 64);
    const float sig = 1.f / (1.f + __expf(-zl));
    const float dz3 = valid ? (float)((double)(sig - yy) * inv_total) : 0.f;
    if (lane < 16 && valid) {
      const double zd = zl;
      loss += fmax(zd, 0.0) - zd * yy + log1p(exp(-fabs(zd)));
    }
    gb3 += (q == 0) ? dz3 : 0.f;
    // layer 3: dW3[h] += dz3[s] h2[s][h]; dH2^T[h][s] = W3[h] dz3[s]; dZ2 = dH2 * (z2 > 0)
    f32x4 dz2[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int h = 16 * ot + 4 * q + i;
        gW3[ot][i] += bf2f((uint16_t)t.h2[ot][i]) * dz3;
        const float d = bf2f(m.W3b[h]) * dz3;
        dz2[ot][i] = t.z2[ot][i] > 0.f ? d : 0.f;
        gb2[ot][i] += dz2[ot][i];
      }
    }
    // dH1^T = W2^T dZ2^T: A = W2^T rows (in) 16 mt + r, cols (out) 16 kt + 4q + i
    bf16x4 bdz2[4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int i = 0; i < 4; ++i) bdz2[kt][i] = (short)f2bf(dz2[kt][i]);
    f32x4 dz1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        bf16x4 a;
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = (short)m.W2b[(16 * kt + 4 * q + i) * kH + 16 * mt + r];
        d = mfma16(a, bdz2[kt], d);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dz1[mt][i] = t.z1[mt][i] > 0.f ? d[i] : 0.f;
        gb1[mt][i] += dz1[mt][i];
      }
    }
    // dW2 = dZ2^T H1: A = dZ2^T [out][sample], B = H1 [sample][in], via LDS
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        s_dz[wave][16 * t4 + 4 * q + i][r] = (uint16_t)bdz2[t4][i];
        s_act[wave][16 * t4 + 4 * q + i][r] = (uint16_t)t.h1[t4][i];
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
      bf16x4 a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (short)s_dz[wave][16 * ot + r][4 * q + i];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        bf16x4 b;
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = (short)s_act[wave][16 * nt + r][4 * q + i];
        gW2[ot][nt] = mfma16(a, b, gW2[ot][nt]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // dW1 = dZ1^T X: A = dZ1^T [hidden][sample] via LDS, B = X [sample][feature]
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
      for (int i = 0; i < 4; ++i) s_dz[wave][16 * t4 + 4 * q + i][r] = f2bf(dz1[t4][i]);
    // X [sample][feature] in LDS rows 0..15 of s_act: row = sample, columns 0..2
    if (q == 0) {
      s_act[wave][r][0] = f2bf(x0);
      s_act[wave][r][1] = f2bf(x1);
      s_act[wave][r][2] = f2bf(x2);
#pragma unroll
      for (int c = 3; c < 16; ++c) s_act[wave][r][c] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    bf16x4 bxs;  // B[k = sample 4q + i][n = feature r]
#pragma unroll
    for (int i = 0; i < 4; ++i) bxs[i] = (short)s_act[wave][4 * q + i][r];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      bf16x4 a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (short)s_dz[wave][16 * mt + r][4 * q + i];
      gW1[mt] = mfma16(a, bxs, gW1[mt]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  // per-wave partials: reduce the per-lane bias / W3 sums over the 16 samples
  // (lanes r = 0..15 of each group q)
  float* out = part + ((uint64_t)blockIdx.x * 4 + wave) * kNParams;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v1 = gb1[a][i], v2 = gb2[a][i], v3 = gW3[a][i];
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) {
        v1 += __shfl_xor(v1, o, 64);
        v2 += __shfl_xor(v2, o, 64);
        v3 += __shfl_xor(v3, o, 64);
      }
      if (r == 0) {
        const int h = 16 * a + 4 * q + i;
        out[oB1 + h] = v1;
        out[oB2 + h] = v2;
        out[oW3 + h] = v3;
      }
    }
  // dW2 tile (ot, nt): lane holds rows (out) 16 ot + 4q + i, column (in) 16 nt + r
#pragma unroll
  for (int ot = 0; ot < 4; ++ot)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[oW2 + (16 * ot + 4 * q + i) * kH + 16 * nt + r] = gW2[ot][nt][i];
  // dW1 tile mt: rows 16 mt + 4q + i, column (feature) r < 3
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (r < 3) out[oW1 + (16 * mt + 4 * q + i) * kIn + r] = gW1[mt][i];
  float b3 = gb3;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) b3 += __shfl_xor(b3, o, 64);
  // gb3 was accumulated on the 16 lanes of group 0 only
  if (lane == 0) out[oB3] = b3;
  double l = loss;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
  if (lane == 0) part_loss[(uint64_t)blockIdx.x * 4 + wave] = l;
}

// Sum of per-wave partials in a fixed order (deterministic).
__global__ void k_grad_reduce(const float* part, const double* part_loss, uint32_t nparts, float* grad,
                              double* loss) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (uint32_t)kNParams) {
    double s = 0.0;
    for (uint32_t p = 0; p < nparts; ++p) s += part[(uint64_t)p * kNParams + i];
    grad[i] = (float)s;
  }
  if (i == 0 && loss) {
    double s = 0.0;
    for (uint32_t p = 0; p < nparts; ++p) s += part_loss[p];
    *loss = s;
  }
}

// Adam step on the FP32 master weights, then refresh the BF16 copies.
__global__ void k_adam(float* w, float* mom1, float* mom2, const float* g, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint32_t)kNParams) return;
  float gi = g[i];
  float m = b1 * mom1[i] + (1.f - b1) * gi;
  float v = b2 * mom2[i] + (1.f - b2) * gi * gi;
  mom1[i] = m;
  mom2[i] = v;
  w[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

__global__ void k_pack(const float* w, uint16_t* W1b, uint16_t* W2b, uint16_t* W3b) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (uint32_t)(kH * 4)) {
    const uint32_t h = i / 4, c = i % 4;
    W1b[i] = c < 3 ? f2bf(w[oW1 + h * kIn + c]) : (uint16_t)0;
  }
  if (i < (uint32_t)(kH * kH)) W2b[i] = f2bf(w[oW2 + i]);
  if (i < (uint32_t)kH) W3b[i] = f2bf(w[oW3 + i]);
}

}  // namespace daic

using namespace daic;

// ---------------------------------------------------------------------------
// Model object
// ---------------------------------------------------------------------------
struct daic_sched_model {
  float* w = nullptr;       // FP32 master [kNParams]
  float* m1 = nullptr;      // Adam moments
  float* m2 = nullptr;
  uint16_t* W1b = nullptr;  // BF16 copies
  uint16_t* W2b = nullptr;
  uint16_t* W3b = nullptr;
  float fmean[3] = {0, 0, 0};  // feature standardization
  float fstd[3] = {1, 1, 1};
  uint64_t adam_t = 0;
  uint64_t version = 0;        // bumped on every change of parameters or scales
  MlpDev dev() const {
    MlpDev m;
    m.W1b = W1b;
    m.W2b = W2b;
    m.W3b = W3b;
    m.b1 = w + oB1;
    m.b2 = w + oB2;
    m.b3 = w + oB3;
    return m;
  }
};

namespace daic {

static daic_status model_pack(daic_sched_model* m, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((kH * kH + 255) / 256), dim3(256), 0, s, m->w, m->W1b, m->W2b, m->W3b);
  DAIC_HIP(hipGetLastError());
  return DAIC_OK;
}

// Gradient of the mean loss over N samples already on the device.
static daic_status model_grad(daic_sched_model* m, const float* dx, const float* dy, uint64_t N, double total,
                              float* dgrad, double* dloss, float* part, double* part_loss, uint32_t blocks,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), 0, s, m->dev(), dx, dy, N, 1.0 / total, part, part_loss);
  hipLaunchKernelGGL(k_grad_reduce, dim3((kNParams + 255) / 256), dim3(256), 0, s, part, part_loss, blocks * 4,
                     dgrad, dloss);
  DAIC_HIP(hipGetLastError());
  return DAIC_OK;
}

constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;

// One Adam step (Kingma and Ba 2015) with the gradient already in dgrad:
// moments and FP32 master weights updated, then the BF16 copies refreshed.
static daic_status adam_apply(daic_sched_model* m, const float* dgrad, float lr, hipStream_t s) {
  m->adam_t += 1;
  m->version += 1;
  const float bc1 = 1.f - std::pow(kAdamB1, (float)m->adam_t);
  const float bc2 = 1.f - std::pow(kAdamB2, (float)m->adam_t);
  hipLaunchKernelGGL(k_adam, dim3((kNParams + 255) / 256), dim3(256), 0, s, m->w, m->m1, m->m2, dgrad, lr, kAdamB1,
                     kAdamB2, kAdamEps, bc1, bc2);
  DAIC_HIP(hipGetLastError());
  return model_pack(m, s);
}

// Serialized model: magic, version, parameter count, Adam step count, the
// feature standardization and the FP32 master weights with both Adam moments.
constexpr char kModelMagic[8] = {'D', 'A', 'I', 'C', 'S', 'C', 'H', '1'};
constexpr uint32_t kModelVersion = 1;
constexpr size_t kModelHeader = 8 + 4 + 4 + 8 + 6 * 4;
constexpr size_t kModelBytes = kModelHeader + 3 * (size_t)kNParams * 4;

}  // namespace daic

extern "C" {

daic_status daic_sched_model_create(const float* params, uint64_t seed, daic_sched_model** out) {
  if (!out) return fail(DAIC_E_INVALID, "out is null");
  *out = nullptr;
  std::unique_ptr<daic_sched_model> m(new daic_sched_model());
  std::vector<float> w(kNParams, 0.0f);
  if (params) {
    std::memcpy(w.data(), params, sizeof(float) * kNParams);
  } else {
    // He-style uniform initialization from a SplitMix64 stream
    uint64_t st = seed;
    auto next = [&]() {
      st += 0x9E3779B97F4A7C15ull;
      uint64_t z = st;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int off, int count, int fan_in) {
      const double lim = std::sqrt(6.0 / fan_in);
      for (int i = 0; i < count; ++i) w[off + i] = (float)((2.0 * next() - 1.0) * lim);
    };
    fill(oW1, kH * kIn, kIn);
    fill(oW2, kH * kH, kH);
    fill(oW3, kH, kH);
  }
  DAIC_HIP(hipMalloc(&m->w, kNParams * 4));
  DAIC_HIP(hipMalloc(&m->m1, kNParams * 4));
  DAIC_HIP(hipMalloc(&m->m2, kNParams * 4));
  DAIC_HIP(hipMalloc(&m->W1b, kH * 4 * 2));
  DAIC_HIP(hipMalloc(&m->W2b, kH * kH * 2));
  DAIC_HIP(hipMalloc(&m->W3b, kH * 2));
  DAIC_HIP(hipMemcpy(m->w, w.data(), kNParams * 4, hipMemcpyHostToDevice));
  DAIC_HIP(hipMemset(m->m1, 0, kNParams * 4));
  DAIC_HIP(hipMemset(m->m2, 0, kNParams * 4));
  daic_status rc = model_pack(m.get(), nullptr);
  if (rc) return rc;
  DAIC_HIP(hipDeviceSynchronize());
  *out = m.release();
  return DAIC_OK;
}

void daic_sched_destroy(daic_sched_model* m) {
  if (!m) return;
  for (void* q : {(void*)m->w, (void*)m->m1, (void*)m->m2, (void*)m->W1b, (void*)m->W2b, (void*)m->W3b})
    if (q) (void)hipFree(q);
  delete m;
}

daic_status daic_sched_model_get(const daic_sched_model* m, float* params, float* feat_mean, float* feat_std) {
  if (!m || !params) return fail(DAIC_E_INVALID, "null argument");
  DAIC_HIP(hipMemcpy(params, m->w, kNParams * 4, hipMemcpyDeviceToHost));
  if (feat_mean) std::memcpy(feat_mean, m->fmean, sizeof m->fmean);
  if (feat_std) std::memcpy(feat_std, m->fstd, sizeof m->fstd);
  return DAIC_OK;
}

daic_status daic_sched_model_set_features(daic_sched_model* m, const float* feat_mean, const float* feat_std) {
  if (!m || !feat_mean || !feat_std) return fail(DAIC_E_INVALID, "null argument");
  for (int i = 0; i < 3; ++i)
    if (!(feat_std[i] > 0.f)) return fail(DAIC_E_INVALID, "feature scales must be positive");
  std::memcpy(m->fmean, feat_mean, sizeof m->fmean);
  std::memcpy(m->fstd, feat_std, sizeof m->fstd);
  m->version += 1;
  return DAIC_OK;
}

daic_status daic_mlp_forward(const daic_sched_model* m, const float* x, uint64_t N, float* logits) {
  if (!m || (N && (!x || !logits))) return fail(DAIC_E_INVALID, "null argument");
  if (N == 0) return DAIC_OK;
  float *dx = nullptr, *dl = nullptr;
  DAIC_HIP(hipMalloc(&dx, N * 3 * 4));
  DAIC_HIP(hipMalloc(&dl, N * 4));
  hipError_t e = hipMemcpy(dx, x, N * 3 * 4, hipMemcpyHostToDevice);
  uint32_t blocks = (uint32_t)std::min<uint64_t>(4096, (N + 63) / 64);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, nullptr, m->dev(), dx, N, dl);
    e = hipMemcpy(logits, dl, N * 4, hipMemcpyDeviceToHost);
  }
  (void)hipFree(dx);
  (void)hipFree(dl);
  if (e != hipSuccess) return fail(DAIC_E_DEVICE, "mlp forward: %s", hipGetErrorString(e));
  return DAIC_OK;
}

daic_status daic_mlp_grad(const daic_sched_model* m, const float* x, const float* y, uint64_t N, float* grad,
                          double* loss) {
  if (!m || !grad || (N && (!x || !y))) return fail(DAIC_E_INVALID, "null argument");
  if (N == 0) return fail(DAIC_E_INVALID, "no samples");
  float *dx = nullptr, *dy = nullptr, *dg = nullptr, *part = nullptr;
  double *dl = nullptr, *pl = nullptr;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (N + 63) / 64);
  DAIC_HIP(hipMalloc(&dx, N * 3 * 4));
  DAIC_HIP(hipMalloc(&dy, N * 4));
  DAIC_HIP(hipMalloc(&dg, kNParams * 4));
  DAIC_HIP(hipMalloc(&dl, 8));
  DAIC_HIP(hipMalloc(&part, (size_t)blocks * 4 * kNParams * 4));
  DAIC_HIP(hipMalloc(&pl, (size_t)blocks * 4 * 8));
  hipError_t e = hipMemcpy(dx, x, N * 3 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dy, y, N * 4, hipMemcpyHostToDevice);
  daic_status rc = DAIC_OK;
  if (e == hipSuccess) {
    rc = model_grad(const_cast<daic_sched_model*>(m), dx, dy, N, (double)N, dg, dl, part, pl, blocks, nullptr);
    if (rc == DAIC_OK) e = hipMemcpy(grad, dg, kNParams * 4, hipMemcpyDeviceToHost);
    if (rc == DAIC_OK && e == hipSuccess && loss) {
      double l = 0;
      e = hipMemcpy(&l, dl, 8, hipMemcpyDeviceToHost);
      *loss = l / (double)N;
    }
  }
  for (void* q : {(void*)dx, (void*)dy, (void*)dg, (void*)dl, (void*)part, (void*)pl}) (void)hipFree(q);
  if (rc) return rc;
  if (e != hipSuccess) return fail(DAIC_E_DEVICE, "mlp grad: %s", hipGetErrorString(e));
  return DAIC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Inference on the problem state, trace capture and training.
// ---------------------------------------------------------------------------
namespace daic {

struct FeatNorm {
  float mean[3];
  float inv_std[3];
};

__global__ void k_indeg(const uint32_t* col, uint64_t m, uint32_t* indeg) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (; i < m; i += st) atomicAdd(&indeg[col[i]], 1u);
}

// Raw features of vertex j: [log2 priority, log2((1 + indeg) / (1 + outdeg)),
// min(rounds since the last update, 64) / 64]; false when j is not pending.
// last_upd holds 1 + the round of the last update (0: never updated), so a
// vertex never updated counts as updated in round -1.
template <int ST, typename RowT>
__device__ __forceinline__ bool vertex_features(const KArgs& a, const uint32_t* indeg, const uint32_t* last_upd,
                                                uint32_t round, uint64_t j, float (&f)[3], float& pr,
                                                uint32_t& since) {
  using S = typename Tr<ST>::S;
  const S v = static_cast<const S*>(a.v)[j];
  const S dv = static_cast<const S*>(a.dv)[j];
  const auto k = prio_key<ST>(v, dv);
  if (k == 0) return false;
  const float p = prio_value<ST>(v, dv);
  const uint64_t od = row_at<RowT>(a.row, j + 1) - row_at<RowT>(a.row, j);
  since = round + 1u - last_upd[j];
  f[0] = log2f(p + 1e-30f);
  f[1] = log2f((1.0f + (float)indeg[j]) / (1.0f + (float)od));
  f[2] = (float)min(since, 64u) * (1.0f / 64.0f);
  pr = p;
  return true;
}

// The network held in registers for the whole scoring kernel: this lane's
// A-operand fragments and the biases of the hidden units whose outputs it
// holds. Layers 2 and 3 use the 16x16x32 BF16 MFMA: in step s (s = 0, 1)
// lane (q, r) supplies 8 products over the hidden units 32 s + 4 q + i and
// 32 s + 16 + 4 q + i (i = 0..3), which are exactly the units of the two
// layer outputs (tiles 2 s and 2 s + 1) the lane already holds; A and B use
// the same assignment, so the sum covers every unit once.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef short i16x8v __attribute__((ext_vector_type(8)));
struct MlpRegs {
  bf16x4 w1[4];      // layer 1, output tile mt: W1 row 16 mt + r, inputs 0..3 (lanes q = 0)
  i16x8v w2[4][2];   // layer 2, output tile ot, step s: W2 row 16 ot + r at the units above
  i16x8v w3[2];      // layer 3, step s: W3 at the units above (lanes r = 0)
  f32x4 b1[4], b2[4];
  float b3;
};

__device__ __forceinline__ uint32_t mlp_unit(int s, uint32_t q, int j) {
  return 32 * s + (j < 4 ? 4 * q + j : 16 + 4 * q + (j - 4));
}

__device__ __forceinline__ void mlp_regs(const MlpDev& m, MlpRegs& R) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t q = lane >> 4, r = lane & 15;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R.w1[t][i] = q == 0 ? (short)m.W1b[(16 * t + r) * 4 + i] : (short)0;
      R.b1[t][i] = m.b1[16 * t + 4 * q + i];
      R.b2[t][i] = m.b2[16 * t + 4 * q + i];
    }
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int j = 0; j < 8; ++j) R.w2[t][st][j] = (short)m.W2b[(16 * t + r) * kH + mlp_unit(st, q, j)];
  }
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int j = 0; j < 8; ++j) R.w3[st][j] = r == 0 ? (short)m.W3b[mlp_unit(st, q, j)] : (short)0;
  R.b3 = m.b3[0];
}

__device__ __forceinline__ f32x4 mfma32(i16x8v a, i16x8v b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a), __builtin_bit_cast(bf16x8v, b), c,
                                                 0, 0, 0);
}

// BF16 of max(z, 0) for the four elements of an MFMA output: a packed
// round-to-nearest-even conversion of each pair, then the ReLU as a packed
// 16-bit integer max with 0 on the BF16 bits (a negative BF16 is a negative
// int16, a non-negative one keeps its order), which equals rounding max(z, 0).
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef short i16x2v __attribute__((ext_vector_type(2)));
typedef short i16x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bf16x4 relu_bf16(f32x4 z) {
  const f32x2v z01 = {z[0], z[1]}, z23 = {z[2], z[3]};
  const i16x2v zero = {0, 0};
  const i16x2v lo = __builtin_elementwise_max(__builtin_bit_cast(i16x2v, __builtin_convertvector(z01, bf16x2v)), zero);
  const i16x2v hi = __builtin_elementwise_max(__builtin_bit_cast(i16x2v, __builtin_convertvector(z23, bf16x2v)), zero);
  return __builtin_bit_cast(bf16x4, __builtin_shufflevector(lo, hi, 0, 1, 2, 3));
}

// Logit of the 16 samples of one tile (lane r of q = 0 ends with sample r's;
// bx: the tile's B operand of layer 1, sample r's inputs in lane r, q = 0).
__device__ __forceinline__ float tile_logit(const MlpRegs& R, bf16x4 bx) {
  bf16x4 h1[4], h2[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) h1[mt] = relu_bf16(mfma16(R.w1[mt], bx, R.b1[mt]));
  const i16x8v g0 = __builtin_shufflevector(__builtin_bit_cast(i16x4v, h1[0]), __builtin_bit_cast(i16x4v, h1[1]),
                                            0, 1, 2, 3, 4, 5, 6, 7);
  const i16x8v g1 = __builtin_shufflevector(__builtin_bit_cast(i16x4v, h1[2]), __builtin_bit_cast(i16x4v, h1[3]),
                                            0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) h2[ot] = relu_bf16(mfma32(R.w2[ot][1], g1, mfma32(R.w2[ot][0], g0, R.b2[ot])));
  const i16x8v k0 = __builtin_shufflevector(__builtin_bit_cast(i16x4v, h2[0]), __builtin_bit_cast(i16x4v, h2[1]),
                                            0, 1, 2, 3, 4, 5, 6, 7);
  const i16x8v k1 = __builtin_shufflevector(__builtin_bit_cast(i16x4v, h2[2]), __builtin_bit_cast(i16x4v, h2[3]),
                                            0, 1, 2, 3, 4, 5, 6, 7);
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  const f32x4 z = mfma32(R.w3[1], k1, mfma32(R.w3[0], k0, zero));
  return z[0] + R.b3;
}

// Selection multiplier of every vertex: sigmoid(network score) for pending
// vertices, a very large value for pending vertices not updated for 64 rounds
// (no vertex is starved), 0 otherwise. A wavefront takes 64 vertices at a
// time (one per lane for the feature loads) and runs them as four 16-sample
// MFMA tiles with the network in registers; 64 vertices without a pending
// one are skipped.
template <int ST, typename RowT>
__global__ __launch_bounds__(256) void k_score(KArgs a, MlpDev m, FeatNorm fn, const uint32_t* indeg,
                                               const uint32_t* last_upd, float* score) {
  if (ctl_halted(a.ctl) || !a.ctl->use_score) return;  // no multipliers for an exact round
  const uint32_t round = (uint32_t)a.ctl->rounds;
  const uint32_t lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
  const uint64_t waves = (uint64_t)gridDim.x * 4;
  MlpRegs R;
  mlp_regs(m, R);
  for (uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c * 64 < a.n; c += waves) {
    const uint64_t j = c * 64 + lane;
    float f[3] = {0.f, 0.f, 0.f}, pr = 0.f;
    uint32_t since = 0;
    bool pend = false;
    if (j < a.n) pend = vertex_features<ST, RowT>(a, indeg, last_upd, round, j, f, pr, since);
    float x[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) x[i] = pend ? (f[i] - fn.mean[i]) * fn.inv_std[i] : 0.f;
    float logit = 0.f;
    if (__ballot(pend) != 0) {  // wave-uniform; the four tiles are independent chains
      float lt[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float y0 = __shfl(x[0], 16 * t + r, 64), y1 = __shfl(x[1], 16 * t + r, 64);
        const float y2 = __shfl(x[2], 16 * t + r, 64);
        bf16x4 bx;
        bx[0] = q == 0 ? __builtin_bit_cast(short, (__bf16)y0) : (short)0;
        bx[1] = q == 0 ? __builtin_bit_cast(short, (__bf16)y1) : (short)0;
        bx[2] = q == 0 ? __builtin_bit_cast(short, (__bf16)y2) : (short)0;
        bx[3] = 0;
        lt[t] = tile_logit(R, bx);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float v = __shfl(lt[t], r, 64);  // sample r of tile t, from lane r
        if (q == (uint32_t)t) logit = v;
      }
    }
    if (j < a.n) score[j] = pend ? (since >= 64 ? 1099511627776.0f : 1.f / (1.f + __expf(-logit))) : 0.f;
  }
}

// Trace capture: S sampled vertices per round.
struct TraceDev {
  uint32_t* vid;   // [R][S]
  float* feat;     // [R][S][3]
  float* p0;       // [R][S] priority when sampled (0: not pending)
  float* maxp;     // [R][S] largest priority over the following rounds
  uint8_t* sel;    // [R][S] updated in the sampled round
};

template <int ST, typename RowT>
__global__ void k_trace_sample(KArgs a, const uint32_t* indeg, const uint32_t* last_upd, TraceDev td,
                               uint64_t seed, uint32_t S, uint32_t slot) {
  const uint32_t round = (uint32_t)a.ctl->rounds;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) {
    const uint64_t j = splitmix64_at(seed, (uint64_t)slot * S + i) % a.n;
    float f[3] = {0.f, 0.f, 0.f}, pr = 0.f;
    uint32_t since = 0;
    const bool pend = vertex_features<ST, RowT>(a, indeg, last_upd, round, j, f, pr, since);
    const uint64_t o = (uint64_t)slot * S + i;
    td.vid[o] = (uint32_t)j;
    td.feat[o * 3] = f[0];
    td.feat[o * 3 + 1] = f[1];
    td.feat[o * 3 + 2] = f[2];
    td.p0[o] = pend ? pr : 0.f;
    td.maxp[o] = 0.f;
    td.sel[o] = 0;
  }
}

// After round `slot`: which samples were updated in it (pending when sampled
// and claimed by the round, which stored slot + 1).
__global__ void k_trace_selected(const uint32_t* last_upd, TraceDev td, uint32_t S, uint32_t slot) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) {
    const uint64_t o = (uint64_t)slot * S + i;
    td.sel[o] = (td.p0[o] > 0.f && last_upd[td.vid[o]] == slot + 1u) ? 1 : 0;
  }
}

// Before a round: fold the current priority into the window maximum of the
// samples of slots [first, last).
template <int ST>
__global__ void k_trace_window(KArgs a, TraceDev td, uint64_t first, uint64_t last) {
  using S = typename Tr<ST>::S;
  for (uint64_t o = first + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < last;
       o += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = td.vid[o];
    const S v = static_cast<const S*>(a.v)[j];
    const S dv = static_cast<const S*>(a.dv)[j];
    const auto k = prio_key<ST>(v, dv);
    float p = prio_value<ST>(v, dv);
    if (k == 0) p = 0.f;
    td.maxp[o] = fmaxf(td.maxp[o], p);
  }
}

template <int ST, typename RowT>
struct LearnedImpl {
  static void score(daic_problem* p, const daic_sched_model* m, const FeatNorm& fn, hipStream_t s) {
    const uint64_t tiles = (p->a.n + 15) / 16;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((tiles + 3) / 4, 8192));
    hipLaunchKernelGGL((k_score<ST, RowT>), dim3(blocks), dim3(256), 0, s, p->a, m->dev(), fn, p->indeg,
                       p->last_upd, p->score);
  }
  static void sample(daic_problem* p, const TraceDev& td, uint64_t seed, uint32_t S, uint32_t slot, hipStream_t s) {
    hipLaunchKernelGGL((k_trace_sample<ST, RowT>), dim3((S + 255) / 256), dim3(256), 0, s, p->a, p->indeg,
                       p->last_upd, td, seed, S, slot);
  }
  static void window(daic_problem* p, const TraceDev& td, uint64_t first, uint64_t last, hipStream_t s) {
    if (last <= first) return;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (last - first + 255) / 256);
    hipLaunchKernelGGL(k_trace_window<ST>, dim3(blocks), dim3(256), 0, s, p->a, td, first, last);
  }
};

struct LearnedOps {
  void (*score)(daic_problem*, const daic_sched_model*, const FeatNorm&, hipStream_t);
  void (*sample)(daic_problem*, const TraceDev&, uint64_t, uint32_t, uint32_t, hipStream_t);
  void (*window)(daic_problem*, const TraceDev&, uint64_t, uint64_t, hipStream_t);
};

template <int ST>
static LearnedOps lops_row(const daic_problem* p) {
  if (p->g->dev.row32)
    return LearnedOps{&LearnedImpl<ST, uint32_t>::score, &LearnedImpl<ST, uint32_t>::sample,
                      &LearnedImpl<ST, uint32_t>::window};
  return LearnedOps{&LearnedImpl<ST, uint64_t>::score, &LearnedImpl<ST, uint64_t>::sample,
                    &LearnedImpl<ST, uint64_t>::window};
}

static LearnedOps learned_ops(const daic_problem* p) {
  switch (p->st) {
    case ST_F64: return lops_row<ST_F64>(p);
    case ST_F32: return lops_row<ST_F32>(p);
    case ST_F32K: return lops_row<ST_F32K>(p);
    case ST_U32: return lops_row<ST_U32>(p);
    case ST_F64MIN: return lops_row<ST_F64MIN>(p);
    default: return lops_row<ST_I32>(p);
  }
}

static FeatNorm norm_of(const daic_sched_model* m) {
  FeatNorm fn;
  for (int i = 0; i < 3; ++i) {
    fn.mean[i] = m->fmean[i];
    fn.inv_std[i] = 1.0f / m->fstd[i];
  }
  return fn;
}

// Per-vertex arrays of the learned scheduler; the update rounds are reset.
static daic_status learned_arrays(daic_problem* p, hipStream_t s) {
  const uint64_t n = p->g->dev.n, m = p->g->dev.m;
  if (!p->learned_ready) {
    DAIC_HIP(hipMalloc(&p->last_upd, std::max<uint64_t>(n, 1) * 4));
    p->allocs.push_back(p->last_upd);
    DAIC_HIP(hipMalloc(&p->indeg, std::max<uint64_t>(n, 1) * 4));
    p->allocs.push_back(p->indeg);
    DAIC_HIP(hipMalloc(&p->score, std::max<uint64_t>(n, 1) * 4));
    p->allocs.push_back(p->score);
    DAIC_HIP(hipMemsetAsync(p->indeg, 0, n * 4, s));
    if (m) {
      const uint32_t blocks = (uint32_t)std::min<uint64_t>(8192, (m + 255) / 256);
      hipLaunchKernelGGL(k_indeg, dim3(blocks), dim3(256), 0, s, p->g->dev.col, m, p->indeg);
    }
    p->learned_ready = true;
  }
  DAIC_HIP(hipMemsetAsync(p->last_upd, 0, n * 4, s));
  p->a.last_upd = p->last_upd;
  return DAIC_OK;
}

daic_status learned_prepare(daic_problem* p, const daic_sched_model* model, hipStream_t s) {
  if (!model) return fail(DAIC_E_INVALID, "LEARNED needs a model");
  return learned_arrays(p, s);
}

daic_status learned_scores_array(daic_problem* p, const daic_sched_model* model, const float** score) {
  if (!model || !p->score) return fail(DAIC_E_INVALID, "LEARNED needs a model and its prepared arrays");
  *score = p->score;
  return DAIC_OK;
}

void learned_scores_enqueue(daic_problem* p, const daic_sched_model* model, hipStream_t s) {
  learned_ops(p).score(p, model, norm_of(model), s);
}

uint64_t learned_model_version(const daic_sched_model* model) { return model ? model->version : 0; }

}  // namespace daic

// Host-side trace: features and labels of the vertices updated in the traced
// rounds, with the windows of H rounds that decide their labels.
struct daic_trace {
  std::vector<float> x;  // [N][3] raw features
  std::vector<float> y;  // [N]
  std::vector<uint32_t> vid;    // [N] vertex of each sample (recorded traces)
  std::vector<uint32_t> round;  // [N] round of each sample (recorded traces)
  uint64_t rounds = 0;
  uint64_t sampled = 0;
  int kind = 0;          // 0 sum, 1 min, 2 max
};

extern "C" {

daic_status daic_sched_score(daic_problem* p, const daic_sched_model* model, float* score_out) {
  if (!p || !model || !score_out) return fail(DAIC_E_INVALID, "null argument");
  const uint64_t n = p->g->dev.n;
  if (n == 0) return DAIC_OK;
  hipStream_t s = p->own_stream;
  daic_status rc = learned_arrays(p, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, p->a.ctl, 0.0, ~0ull);
  learned_ops(p).score(p, model, norm_of(model), s);
  hipError_t e = hipMemcpyAsync(score_out, p->score, n * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(DAIC_E_DEVICE, "sched_score: %s", hipGetErrorString(e));
  return DAIC_OK;
}

// Runs exact top-k rounds (opts: sched TOPK_EXACT, q, eps, max_rounds) from
// the problem's current state to the stop rule, sampling S vertices per round.
// A vertex updated in round t is labelled 1 ("update now") unless within the
// next H rounds its priority reaches half its priority at t (sum problems) or
// it becomes pending again at all (min/max problems): then its update was
// premature and the label is 0.
daic_status daic_trace_record(daic_problem* p, const daic_run_opts* o, uint32_t samples_per_round,
                              uint32_t horizon, daic_trace** out) {
  if (!p || !o || !out) return fail(DAIC_E_INVALID, "null argument");
  *out = nullptr;
  daic_status rc = check_opts(p, o);
  if (rc) return rc;
  if (o->sched != DAIC_SCHED_TOPK_EXACT) return fail(DAIC_E_INVALID, "traces come from exact top-k runs");
  apply_run_opts(p, o);
  if (samples_per_round == 0 || samples_per_round > (1u << 20) || horizon == 0 || horizon > 64)
    return fail(DAIC_E_INVALID, "samples_per_round in 1..2^20 and horizon in 1..64");
  const uint64_t n = p->g->dev.n;
  std::unique_ptr<daic_trace> tr(new daic_trace());
  tr->kind = p->op == DAIC_SUM ? 0 : (p->op == DAIC_MIN ? 1 : 2);
  if (n == 0) {
    *out = tr.release();
    return DAIC_OK;
  }
  Ops ops;
  if (!get_ops(p, &ops)) return fail(DAIC_E_UNSUPPORTED, "no kernel for this combination");
  hipStream_t s = o->hip_stream ? static_cast<hipStream_t>(o->hip_stream) : p->own_stream;
  rc = learned_arrays(p, s);
  if (rc) return rc;
  rc = dense_rounds_setup(p, o, s);
  if (rc) return rc;
  const uint32_t S = samples_per_round, H = horizon;
  const uint64_t R = std::min<uint64_t>(o->max_rounds ? o->max_rounds : 4096, 4096);
  TraceDev td{};
  DAIC_HIP(hipMalloc(&td.vid, R * S * 4));
  DAIC_HIP(hipMalloc(&td.feat, R * S * 12));
  DAIC_HIP(hipMalloc(&td.p0, R * S * 4));
  DAIC_HIP(hipMalloc(&td.maxp, R * S * 4));
  DAIC_HIP(hipMalloc(&td.sel, R * S));
  LearnedOps lo = learned_ops(p);
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, p->a.ctl, o->eps, R);
  ops.residual(p, s, 0);
  uint64_t t = 0;
  hipError_t e = hipSuccess;
  for (; t < R; ++t) {
    e = hipMemcpyAsync(p->h_ctl, p->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || p->h_ctl->done || p->h_ctl->stop) break;
    const uint64_t first = t >= H ? (t - H) * S : 0;
    lo.window(p, td, first, t * S, s);
    lo.sample(p, td, o->seed ^ 0x7A3E5C91u, S, (uint32_t)t, s);
    ops.round(p, o, s, nullptr, nullptr);
    hipLaunchKernelGGL(k_trace_selected, dim3((S + 255) / 256), dim3(256), 0, s, p->last_upd, td, S, (uint32_t)t);
  }
  // the state after the last round stands for the start of every later round
  if (e == hipSuccess && t > 0) lo.window(p, td, t >= H ? (t - H) * S : 0, t * S, s);
  std::vector<float> feat, p0, maxp;
  std::vector<uint8_t> sel;
  std::vector<uint32_t> vids;
  if (e == hipSuccess) {
    const uint64_t cnt = t * S;
    feat.resize(cnt * 3);
    p0.resize(cnt);
    maxp.resize(cnt);
    sel.resize(cnt);
    vids.resize(cnt);
    if (cnt) {
      e = hipMemcpy(feat.data(), td.feat, cnt * 12, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(vids.data(), td.vid, cnt * 4, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(p0.data(), td.p0, cnt * 4, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(maxp.data(), td.maxp, cnt * 4, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(sel.data(), td.sel, cnt, hipMemcpyDeviceToHost);
    }
  }
  for (void* q : {(void*)td.vid, (void*)td.feat, (void*)td.p0, (void*)td.maxp, (void*)td.sel}) (void)hipFree(q);
  p->a.last_upd = nullptr;
  if (e != hipSuccess) return fail(DAIC_E_DEVICE, "trace: %s", hipGetErrorString(e));
  // labels from complete windows only
  const bool done = p->h_ctl->done != 0;
  const uint64_t full = done ? t : (t > H ? t - H : 0);
  for (uint64_t r = 0; r < full; ++r)
    for (uint32_t i = 0; i < S; ++i) {
      const uint64_t o2 = r * S + i;
      ++tr->sampled;
      if (!sel[o2]) continue;
      const bool premature = tr->kind == 0 ? (maxp[o2] >= 0.5f * p0[o2]) : (maxp[o2] > 0.f);
      tr->x.insert(tr->x.end(), &feat[o2 * 3], &feat[o2 * 3] + 3);
      tr->y.push_back(premature ? 0.f : 1.f);
      tr->vid.push_back(vids[o2]);
      tr->round.push_back((uint32_t)r);
    }
  tr->rounds = t;
  *out = tr.release();
  return DAIC_OK;
}

daic_status daic_trace_get(const daic_trace* tr, float* x, float* y, uint64_t* n) {
  if (!tr || !n) return fail(DAIC_E_INVALID, "null argument");
  if (x) std::memcpy(x, tr->x.data(), tr->x.size() * 4);
  if (y) std::memcpy(y, tr->y.data(), tr->y.size() * 4);
  *n = tr->y.size();
  return DAIC_OK;
}

void daic_trace_destroy(daic_trace* tr) { delete tr; }

daic_status daic_trace_samples(const daic_trace* tr, uint32_t* vid, uint32_t* round, uint64_t* n) {
  if (!tr || !n) return fail(DAIC_E_INVALID, "null argument");
  *n = tr->vid.size();
  if (vid) std::memcpy(vid, tr->vid.data(), tr->vid.size() * 4);
  if (round) std::memcpy(round, tr->round.data(), tr->round.size() * 4);
  return DAIC_OK;
}

daic_status daic_trace_create(const float* x, const float* y, uint64_t n, daic_trace** out) {
  if (!out || (n && (!x || !y))) return fail(DAIC_E_INVALID, "null argument");
  *out = nullptr;
  for (uint64_t i = 0; i < n; ++i) {
    if (!(y[i] == 0.f || y[i] == 1.f)) return fail(DAIC_E_INVALID, "label %llu is not 0 or 1", (unsigned long long)i);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(x[i * 3 + k])) return fail(DAIC_E_INVALID, "feature %llu is not finite", (unsigned long long)i);
  }
  std::unique_ptr<daic_trace> tr(new daic_trace());
  tr->x.assign(x, x + n * 3);
  tr->y.assign(y, y + n);
  *out = tr.release();
  return DAIC_OK;
}

daic_status daic_sched_step(daic_sched_model* m, const float* x, const float* y, uint64_t N, float lr,
                            float* grad_out, double* loss) {
  if (!m || (N && (!x || !y))) return fail(DAIC_E_INVALID, "null argument");
  if (N == 0) return fail(DAIC_E_INVALID, "no samples");
  if (!(lr > 0.f)) return fail(DAIC_E_INVALID, "lr must be positive");
  float *dx = nullptr, *dy = nullptr, *dg = nullptr, *part = nullptr;
  double *dl = nullptr, *pl = nullptr;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (N + 63) / 64);
  std::vector<void*> bufs;
  auto grab = [&](void** q, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(q, bytes);
    if (e == hipSuccess) bufs.push_back(*q);
    return e;
  };
  hipError_t e = grab((void**)&dx, N * 12);
  if (e == hipSuccess) e = grab((void**)&dy, N * 4);
  if (e == hipSuccess) e = grab((void**)&dg, kNParams * 4);
  if (e == hipSuccess) e = grab((void**)&dl, 8);
  if (e == hipSuccess) e = grab((void**)&part, (size_t)blocks * 4 * kNParams * 4);
  if (e == hipSuccess) e = grab((void**)&pl, (size_t)blocks * 4 * 8);
  if (e == hipSuccess) e = hipMemcpy(dx, x, N * 12, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dy, y, N * 4, hipMemcpyHostToDevice);
  daic_status rc = e == hipSuccess ? DAIC_OK : fail(DAIC_E_DEVICE, "sched_step: %s", hipGetErrorString(e));
  if (rc == DAIC_OK) rc = model_grad(m, dx, dy, N, (double)N, dg, dl, part, pl, blocks, nullptr);
  if (rc == DAIC_OK) rc = adam_apply(m, dg, lr, nullptr);
  if (rc == DAIC_OK && grad_out) {
    e = hipMemcpy(grad_out, dg, kNParams * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(DAIC_E_DEVICE, "sched_step: %s", hipGetErrorString(e));
  }
  if (rc == DAIC_OK && loss) {
    double l = 0;
    e = hipMemcpy(&l, dl, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(DAIC_E_DEVICE, "sched_step: %s", hipGetErrorString(e));
    *loss = l / (double)N;
  }
  if (rc == DAIC_OK) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = fail(DAIC_E_DEVICE, "sched_step: %s", hipGetErrorString(e));
  }
  for (void* q : bufs) (void)hipFree(q);
  return rc;
}

daic_status daic_sched_save(const daic_sched_model* m, void* buf, size_t* len) {
  if (!m || !len) return fail(DAIC_E_INVALID, "null argument");
  if (!buf) {
    *len = kModelBytes;
    return DAIC_OK;
  }
  if (*len < kModelBytes) {
    const size_t have = *len;
    *len = kModelBytes;
    return fail(DAIC_E_INVALID, "buffer of %zu bytes, %zu needed", have, kModelBytes);
  }
  uint8_t* b = static_cast<uint8_t*>(buf);
  const uint32_t ver = kModelVersion, np = (uint32_t)kNParams;
  const uint64_t t = m->adam_t;
  std::memcpy(b, kModelMagic, 8);
  std::memcpy(b + 8, &ver, 4);
  std::memcpy(b + 12, &np, 4);
  std::memcpy(b + 16, &t, 8);
  std::memcpy(b + 24, m->fmean, 12);
  std::memcpy(b + 36, m->fstd, 12);
  float* w = reinterpret_cast<float*>(b + kModelHeader);
  DAIC_HIP(hipMemcpy(w, m->w, kNParams * 4, hipMemcpyDeviceToHost));
  DAIC_HIP(hipMemcpy(w + kNParams, m->m1, kNParams * 4, hipMemcpyDeviceToHost));
  DAIC_HIP(hipMemcpy(w + 2 * kNParams, m->m2, kNParams * 4, hipMemcpyDeviceToHost));
  *len = kModelBytes;
  return DAIC_OK;
}

daic_status daic_sched_load(const void* buf, size_t len, daic_sched_model** out) {
  if (!buf || !out) return fail(DAIC_E_INVALID, "null argument");
  *out = nullptr;
  const uint8_t* b = static_cast<const uint8_t*>(buf);
  if (len < kModelHeader || std::memcmp(b, kModelMagic, 8) != 0) return fail(DAIC_E_INVALID, "not a saved model");
  uint32_t ver, np;
  uint64_t t;
  std::memcpy(&ver, b + 8, 4);
  std::memcpy(&np, b + 12, 4);
  std::memcpy(&t, b + 16, 8);
  if (ver != kModelVersion || np != (uint32_t)kNParams) return fail(DAIC_E_INVALID, "unsupported model version or size");
  if (len != kModelBytes) return fail(DAIC_E_INVALID, "model buffer of %zu bytes, %zu expected", len, kModelBytes);
  float mean[3], sd[3];
  std::memcpy(mean, b + 24, 12);
  std::memcpy(sd, b + 36, 12);
  std::vector<float> w(3 * (size_t)kNParams);
  std::memcpy(w.data(), b + kModelHeader, w.size() * 4);
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(mean[k]) || !(sd[k] > 0.f) || !std::isfinite(sd[k]))
      return fail(DAIC_E_INVALID, "bad feature standardization");
  for (float x : w)
    if (!std::isfinite(x)) return fail(DAIC_E_INVALID, "non-finite parameter");
  daic_sched_model* m = nullptr;
  daic_status rc = daic_sched_model_create(w.data(), 0, &m);
  if (rc) return rc;
  hipError_t e = hipMemcpy(m->m1, w.data() + kNParams, kNParams * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->m2, w.data() + 2 * kNParams, kNParams * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    daic_sched_destroy(m);
    return fail(DAIC_E_DEVICE, "sched_load: %s", hipGetErrorString(e));
  }
  std::memcpy(m->fmean, mean, 12);
  std::memcpy(m->fstd, sd, 12);
  m->adam_t = t;
  *out = m;
  return DAIC_OK;
}

// Trains the model on the union of the traces: features standardized with
// their mean and scale (kept in the model), minibatch Adam on the mean
// BCE-with-logits loss, gradients from the BF16 MFMA kernels.
daic_status daic_sched_train(const daic_trace* const* traces, uint32_t n_traces, const daic_train_opts* to,
                             daic_sched_model* m, daic_train_stats* st) {
  if (!traces || !to || !m) return fail(DAIC_E_INVALID, "null argument");
  std::vector<float> x, y;
  for (uint32_t i = 0; i < n_traces; ++i) {
    if (!traces[i]) return fail(DAIC_E_INVALID, "trace %u is null", i);
    x.insert(x.end(), traces[i]->x.begin(), traces[i]->x.end());
    y.insert(y.end(), traces[i]->y.begin(), traces[i]->y.end());
  }
  const uint64_t N = y.size();
  if (N == 0) return fail(DAIC_E_INVALID, "no samples in the traces");
  // standardization
  double mean[3] = {0, 0, 0}, var[3] = {0, 0, 0};
  for (uint64_t i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) mean[k] += x[i * 3 + k];
  for (int k = 0; k < 3; ++k) mean[k] /= (double)N;
  for (uint64_t i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) var[k] += (x[i * 3 + k] - mean[k]) * (x[i * 3 + k] - mean[k]);
  for (int k = 0; k < 3; ++k) {
    m->fmean[k] = (float)mean[k];
    m->fstd[k] = (float)std::max(1e-6, std::sqrt(var[k] / (double)N));
  }
  m->version += 1;
  // shuffle with a seeded Fisher-Yates on SplitMix64 draws, then standardize
  std::vector<uint64_t> perm(N);
  for (uint64_t i = 0; i < N; ++i) perm[i] = i;
  uint64_t state = to->seed;
  for (uint64_t i = N - 1; i > 0; --i) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    std::swap(perm[i], perm[z % (i + 1)]);
  }
  std::vector<float> xs(N * 3), ys(N);
  double pos = 0;
  for (uint64_t i = 0; i < N; ++i) {
    const uint64_t s0 = perm[i];
    for (int k = 0; k < 3; ++k) xs[i * 3 + k] = (float)((x[s0 * 3 + k] - mean[k]) / m->fstd[k]);
    ys[i] = y[s0];
    pos += y[s0];
  }
  const uint64_t B = std::max<uint64_t>(16, std::min<uint64_t>(to->batch ? to->batch : 65536, N));
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (B + 63) / 64);
  float *dx = nullptr, *dy = nullptr, *dg = nullptr, *part = nullptr;
  double *dl = nullptr, *pl = nullptr;
  DAIC_HIP(hipMalloc(&dx, N * 12));
  DAIC_HIP(hipMalloc(&dy, N * 4));
  DAIC_HIP(hipMalloc(&dg, kNParams * 4));
  DAIC_HIP(hipMalloc(&dl, 8));
  DAIC_HIP(hipMalloc(&part, (size_t)blocks * 4 * kNParams * 4));
  DAIC_HIP(hipMalloc(&pl, (size_t)blocks * 4 * 8));
  DAIC_HIP(hipMemcpy(dx, xs.data(), N * 12, hipMemcpyHostToDevice));
  DAIC_HIP(hipMemcpy(dy, ys.data(), N * 4, hipMemcpyHostToDevice));
  hipStream_t s = nullptr;
  hipEvent_t e0, e1;
  DAIC_HIP(hipEventCreate(&e0));
  DAIC_HIP(hipEventCreate(&e1));
  auto full_loss = [&](double* out_loss) -> daic_status {
    daic_status rc2 = model_grad(m, dx, dy, N, (double)N, dg, dl, part, pl, blocks, s);
    if (rc2) return rc2;
    double l = 0;
    DAIC_HIP(hipMemcpy(&l, dl, 8, hipMemcpyDeviceToHost));
    *out_loss = l / (double)N;
    return DAIC_OK;
  };
  double loss0 = 0, loss1 = 0;
  daic_status rc = full_loss(&loss0);
  DAIC_HIP(hipEventRecord(e0, s));
  const float lr = to->lr > 0 ? to->lr : 1e-3f;
  const uint32_t epochs = to->epochs ? to->epochs : 10;
  for (uint32_t ep = 0; ep < epochs && rc == DAIC_OK; ++ep) {
    for (uint64_t off = 0; off < N && rc == DAIC_OK; off += B) {
      const uint64_t nb = std::min<uint64_t>(B, N - off);
      rc = model_grad(m, dx + off * 3, dy + off, nb, (double)nb, dg, nullptr, part, pl, blocks, s);
      if (rc == DAIC_OK) rc = adam_apply(m, dg, lr, s);
    }
  }
  DAIC_HIP(hipEventRecord(e1, s));
  DAIC_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  DAIC_HIP(hipEventElapsedTime(&ms, e0, e1));
  if (rc == DAIC_OK) rc = full_loss(&loss1);
  for (void* q : {(void*)dx, (void*)dy, (void*)dg, (void*)dl, (void*)part, (void*)pl}) (void)hipFree(q);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (st) {
    st->samples = N;
    st->positive_fraction = pos / (double)N;
    st->loss_first = loss0;
    st->loss_final = loss1;
    st->time_ms = ms;
    st->epochs = epochs;
  }
  return DAIC_OK;
}

}  // extern "C"
