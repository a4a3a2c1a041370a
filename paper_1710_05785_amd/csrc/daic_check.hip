// Check of the fourth condition of DAIC (Sec. 3.1): the initial values must
// satisfy v0_j (+) dv1_j = f(v0)_j, where f is the update function of Eq.
// decompose, f(v)_j = (+)_{i -> j} g_{i,j}(v_i) (+) c_j. The same identity
// holds at every state a run leaves (all messages delivered: the delta of a
// vertex is the (+)-sum of what its in-neighbours' updates sent it since its
// own last update), so the check takes the problem's current state.
//
// f(v) is formed by a push over every edge into per-vertex accumulators
// (FP64 for the sum problems, with a second accumulator of the terms'
// absolute values that scales the tolerance; exact for min and max), then
// each vertex compares. It is a debug path: the accumulators are allocated
// per call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <cstdlib>
#include <limits>
#include <vector>

#include "daic_device.h"
#include "daic_internal.h"
#include "daic_kernels.h"
#include "daic_problem.h"

namespace daic {

struct CheckBuf {
  void* acc;           // sum: double; min U32: uint32; min F64: uint64 bits; max: int32
  double* absacc;      // sum problems: sum of |g(v_i)|
  const void* cst;     // c_j in the state's host element type on the device (double for FP states)
  double* total;       // sum problems: sum over vertices of each vertex's magnitude scale
  unsigned long long* bad;    // [0] mismatches, [1] smallest mismatching vertex,
                              // [2] bits of the largest |lhs - rhs| / scale (sum problems)
};

// Every edge (j -> k) adds g_jk(v_j) into the accumulator of k.
template <int ST, int G, typename RowT>
__global__ __launch_bounds__(256) void k_check_push(KArgs a, CheckBuf cb) {
  using S = typename Tr<ST>::S;
  const S* v = static_cast<const S*>(a.v);
  for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < a.n; j += (uint64_t)gridDim.x * 256) {
    const uint64_t e0 = row_at<RowT>(a.row, j), e1 = row_at<RowT>(a.row, j + 1);
    if constexpr (Tr<ST>::sum) {
      double x = (double)v[j];
      if constexpr (Tr<ST>::kahan) x -= (double)a.c[j];
      double coef;
      if constexpr (G == DAIC_G_DEG_SCALE) coef = e1 > e0 ? a.alpha / (double)(e1 - e0) : 0.0;
      else coef = a.alpha_pv ? (double)static_cast<const S*>(a.alpha_pv)[j] : a.alpha;
      for (uint64_t e = e0; e < e1; ++e) {
        double t = coef * x;
        if constexpr (G == DAIC_G_EDGE_SCALE) t *= (double)static_cast<const S*>(a.w)[e];
        const uint32_t k = a.col[e];
        atomicAdd(&static_cast<double*>(cb.acc)[k], t);
        atomicAdd(&cb.absacc[k], fabs(t));
      }
    } else if constexpr (ST == ST_U32) {
      const uint32_t x = v[j];
      if (x == kInfU32) continue;  // g(infinity) is the identity: nothing sent
      for (uint64_t e = e0; e < e1; ++e) {
        const uint64_t s = (uint64_t)x + static_cast<const uint32_t*>(a.w)[e];
        atomicMin(&static_cast<uint32_t*>(cb.acc)[a.col[e]], s >= kInfU32 ? kInfU32 : (uint32_t)s);
      }
    } else if constexpr (ST == ST_F64MIN) {
      const double x = v[j];
      if (isinf(x)) continue;
      for (uint64_t e = e0; e < e1; ++e) {
        const double m = x + static_cast<const double*>(a.w)[e];
        atomicMin(&static_cast<unsigned long long*>(cb.acc)[a.col[e]], (unsigned long long)__double_as_longlong(m));
      }
    } else {
      const int32_t x = v[j];
      if (x == -1) continue;  // the identity of max
      for (uint64_t e = e0; e < e1; ++e) atomicMax(&static_cast<int32_t*>(cb.acc)[a.col[e]], x);
    }
  }
}

// Magnitude scale of vertex k's identity: |c_k| + sum |g_ik(v_i)| + |v_k| + |dv_k|.
template <int ST>
__device__ __forceinline__ double check_scale(const KArgs& a, const CheckBuf& cb, uint64_t k) {
  using S = typename Tr<ST>::S;
  double vk = (double)static_cast<const S*>(a.v)[k];
  if constexpr (Tr<ST>::kahan) vk -= (double)a.c[k];
  return fabs(static_cast<const double*>(cb.cst)[k]) + cb.absacc[k] + fabs(vk) +
         fabs((double)static_cast<const S*>(a.dv)[k]);
}

// Sum problems: the total of the vertices' scales (its mean sets an absolute
// floor of the tolerance: where the terms of a vertex cancel, the rounding
// left from earlier states is of the size of the state's typical values).
template <int ST>
__global__ __launch_bounds__(256) void k_check_total(KArgs a, CheckBuf cb) {
  if constexpr (Tr<ST>::sum) {
    double t = 0.0;
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < a.n; k += (uint64_t)gridDim.x * 256)
      t += check_scale<ST>(a, cb, k);
    t = block_sum256(t);
    if (threadIdx.x == 0) atomicAdd(cb.total, t);
  }
}

// Every vertex: v_k (+) dv_k against acc_k (+) c_k.
template <int ST>
__global__ __launch_bounds__(256) void k_check_compare(KArgs a, CheckBuf cb, double tol) {
  using S = typename Tr<ST>::S;
  const S* v = static_cast<const S*>(a.v);
  const S* dv = static_cast<const S*>(a.dv);
  for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < a.n; k += (uint64_t)gridDim.x * 256) {
    bool ok;
    if constexpr (Tr<ST>::sum) {
      double vk = (double)v[k];
      if constexpr (Tr<ST>::kahan) vk -= (double)a.c[k];
      const double ck = static_cast<const double*>(cb.cst)[k];
      const double lhs = vk + (double)dv[k];
      const double rhs = static_cast<const double*>(cb.acc)[k] + ck;
      const double scale = check_scale<ST>(a, cb, k) + *cb.total / (double)a.n;
      const double dev = fabs(lhs - rhs);
      ok = dev <= tol * scale;
      if (dev > 0.0) {
        const double rel = scale > 0.0 ? dev / scale : 1.0;
        atomicMax(&cb.bad[2], (unsigned long long)__double_as_longlong(rel));  // non-negative: bits order like values
      }
    } else if constexpr (ST == ST_U32) {
      const uint32_t ck = static_cast<const uint32_t*>(cb.cst)[k];
      const uint32_t lhs = min(v[k], dv[k]);
      const uint32_t rhs = min(static_cast<const uint32_t*>(cb.acc)[k], ck);
      ok = lhs == rhs;
    } else if constexpr (ST == ST_F64MIN) {
      const double ck = static_cast<const double*>(cb.cst)[k];
      const double lhs = fmin(v[k], dv[k]);
      const double rhs = fmin(__longlong_as_double((long long)static_cast<const unsigned long long*>(cb.acc)[k]), ck);
      ok = lhs == rhs;
    } else {
      const int32_t ck = static_cast<const int32_t*>(cb.cst)[k];
      const int32_t lhs = max(v[k], dv[k]);
      const int32_t rhs = max(static_cast<const int32_t*>(cb.acc)[k], ck);
      ok = lhs == rhs;
    }
    if (!ok) {
      atomicAdd(&cb.bad[0], 1ull);
      atomicMin(&cb.bad[1], (unsigned long long)k);
    }
  }
}

template <typename T>
__global__ void k_check_fill(T* p, T val, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256) p[i] = val;
}

template <int ST, int G, typename RowT>
static void check_launch(daic_problem* p, const CheckBuf& cb, double tol, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL((k_check_push<ST, G, RowT>), dim3(grid), dim3(256), 0, s, p->a, cb);
  hipLaunchKernelGGL(k_check_total<ST>, dim3(grid), dim3(256), 0, s, p->a, cb);
  hipLaunchKernelGGL(k_check_compare<ST>, dim3(grid), dim3(256), 0, s, p->a, cb, tol);
}

template <int ST, int G>
static void check_row(daic_problem* p, const CheckBuf& cb, double tol, uint32_t grid, hipStream_t s) {
  if (p->g->dev.row32) check_launch<ST, G, uint32_t>(p, cb, tol, grid, s);
  else check_launch<ST, G, uint64_t>(p, cb, tol, grid, s);
}

static bool check_dispatch(daic_problem* p, const CheckBuf& cb, double tol, uint32_t grid, hipStream_t s) {
  switch (p->st) {
    case ST_F64:
      if (p->gk == DAIC_G_SRC_SCALE) check_row<ST_F64, DAIC_G_SRC_SCALE>(p, cb, tol, grid, s);
      else if (p->gk == DAIC_G_DEG_SCALE) check_row<ST_F64, DAIC_G_DEG_SCALE>(p, cb, tol, grid, s);
      else check_row<ST_F64, DAIC_G_EDGE_SCALE>(p, cb, tol, grid, s);
      return true;
    case ST_F32:
      if (p->gk == DAIC_G_SRC_SCALE) check_row<ST_F32, DAIC_G_SRC_SCALE>(p, cb, tol, grid, s);
      else if (p->gk == DAIC_G_DEG_SCALE) check_row<ST_F32, DAIC_G_DEG_SCALE>(p, cb, tol, grid, s);
      else check_row<ST_F32, DAIC_G_EDGE_SCALE>(p, cb, tol, grid, s);
      return true;
    case ST_F32K:
      if (p->gk == DAIC_G_SRC_SCALE) check_row<ST_F32K, DAIC_G_SRC_SCALE>(p, cb, tol, grid, s);
      else if (p->gk == DAIC_G_DEG_SCALE) check_row<ST_F32K, DAIC_G_DEG_SCALE>(p, cb, tol, grid, s);
      else check_row<ST_F32K, DAIC_G_EDGE_SCALE>(p, cb, tol, grid, s);
      return true;
    case ST_U32: check_row<ST_U32, DAIC_G_EDGE_ADD>(p, cb, tol, grid, s); return true;
    case ST_F64MIN: check_row<ST_F64MIN, DAIC_G_EDGE_ADD>(p, cb, tol, grid, s); return true;
    case ST_I32: check_row<ST_I32, DAIC_G_COPY>(p, cb, tol, grid, s); return true;
  }
  return false;
}

static bool fp_state(int st) { return st == ST_F64 || st == ST_F32 || st == ST_F32K || st == ST_F64MIN; }

daic_status check_init(daic_problem* p, double tol, uint64_t* mismatches, hipStream_t s) {
  const uint64_t n = p->g->dev.n;
  if (mismatches) *mismatches = 0;
  if (!p->cst) return fail(DAIC_E_INVALID, "the fourth-condition check needs the constant c (daic_problem_set_const)");
  if (n == 0) return DAIC_OK;
  const bool sum = p->st == ST_F64 || p->st == ST_F32 || p->st == ST_F32K;
  if (tol <= 0.0) tol = p->st == ST_F64 ? 1e-12 : 1e-5;
  CheckBuf cb{};
  cb.cst = p->cst;
  std::vector<void*> bufs;
  auto grab = [&](void** q, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(q, bytes);
    if (e == hipSuccess) bufs.push_back(*q);
    return e;
  };
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(8192, (n + 255) / 256));
  hipError_t e = grab(&cb.acc, n * 8);
  if (e == hipSuccess && sum) e = grab((void**)&cb.absacc, n * 8);
  if (e == hipSuccess) e = grab((void**)&cb.bad, 24);
  if (e == hipSuccess) e = grab((void**)&cb.total, 8);
  if (e == hipSuccess) {
    if (sum) {
      hipLaunchKernelGGL(k_check_fill<double>, dim3(grid), dim3(256), 0, s, static_cast<double*>(cb.acc), 0.0, n);
      hipLaunchKernelGGL(k_check_fill<double>, dim3(grid), dim3(256), 0, s, cb.absacc, 0.0, n);
    } else if (p->st == ST_U32) {
      hipLaunchKernelGGL(k_check_fill<uint32_t>, dim3(grid), dim3(256), 0, s, static_cast<uint32_t*>(cb.acc), kInfU32, n);
    } else if (p->st == ST_F64MIN) {
      const double inf = std::numeric_limits<double>::infinity();
      unsigned long long bits;
      std::memcpy(&bits, &inf, 8);
      hipLaunchKernelGGL(k_check_fill<unsigned long long>, dim3(grid), dim3(256), 0, s,
                         static_cast<unsigned long long*>(cb.acc), bits, n);
    } else {
      hipLaunchKernelGGL(k_check_fill<int32_t>, dim3(grid), dim3(256), 0, s, static_cast<int32_t*>(cb.acc), -1, n);
    }
    hipLaunchKernelGGL(k_check_fill<unsigned long long>, dim3(1), dim3(256), 0, s, cb.bad, 0ull, 1);
    hipLaunchKernelGGL(k_check_fill<unsigned long long>, dim3(1), dim3(256), 0, s, cb.bad + 1, ~0ull, 1);
    hipLaunchKernelGGL(k_check_fill<unsigned long long>, dim3(1), dim3(256), 0, s, cb.bad + 2, 0ull, 1);
    hipLaunchKernelGGL(k_check_fill<double>, dim3(1), dim3(256), 0, s, cb.total, 0.0, 1);
    check_dispatch(p, cb, tol, grid, s);
    e = hipGetLastError();
  }
  unsigned long long hb[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hb, cb.bad, 24, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (void* q : bufs) (void)hipFree(q);
  if (e != hipSuccess) return fail(DAIC_E_DEVICE, "fourth-condition check: %s", hipGetErrorString(e));
  if (mismatches) *mismatches = hb[0];
  double worst = 0.0;
  std::memcpy(&worst, &hb[2], 8);
  if (hb[0])
    return fail(DAIC_E_INVALID, "v (+) dv != f(v) at %llu vertices (first: %llu; largest deviation %.3g of the "
                "terms' magnitude, tolerance %.3g): the state breaks the fourth condition",
                (unsigned long long)hb[0], (unsigned long long)hb[1], worst, tol);
  (void)fp_state;
  return DAIC_OK;
}

}  // namespace daic

using namespace daic;

extern "C" {

daic_status daic_problem_set_const(daic_problem* p, const void* c) {
  if (!p || !c) return fail(DAIC_E_INVALID, "null argument");
  const uint64_t n = p->g->dev.n;
  const bool fp = p->st == ST_F64 || p->st == ST_F32 || p->st == ST_F32K || p->st == ST_F64MIN;
  const size_t S = fp ? 8 : 4;  // double for FP states, the state's integer type otherwise
  if (!p->cst) {
    void* q = nullptr;
    DAIC_HIP(hipMalloc(&q, std::max<uint64_t>(n, 1) * S));
    p->allocs.push_back(q);
    p->cst = q;
  }
  if (n) DAIC_HIP(hipMemcpy(p->cst, c, n * S, hipMemcpyHostToDevice));
  return DAIC_OK;
}

daic_status daic_problem_check_init(daic_problem* p, double tol, uint64_t* mismatches) {
  if (!p) return fail(DAIC_E_INVALID, "null argument");
  if (!(tol >= 0.0)) return fail(DAIC_E_INVALID, "tol must be >= 0");
  return check_init(p, tol, mismatches, p->own_stream);
}

}  // extern "C"
