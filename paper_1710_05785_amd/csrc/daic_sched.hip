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
// Placeholder hooks of the round loop (replaced once inference is in place).
// ---------------------------------------------------------------------------
namespace daic {
daic_status learned_prepare(daic_problem*, const daic_sched_model*, hipStream_t) {
  return fail(DAIC_E_UNSUPPORTED, "learned scheduler not available");
}
daic_status learned_scores(daic_problem*, const daic_sched_model*, hipStream_t, const float**) {
  return fail(DAIC_E_UNSUPPORTED, "learned scheduler not available");
}
void learned_after_round(daic_problem*, hipStream_t) {}
}  // namespace daic
