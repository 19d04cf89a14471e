// Learned degree per tent: tent features, a small MLP with BF16 weights and
// FP32 accumulation (forward, backward, Adam), and the degree choice.
//
// The network maps kFeat tent features to predictions of log(eta_T(p)) for
// p = 2..8, eta_T being the energy of the jump between the tent solution of
// degree p and the incoming trace on the bottom facets (computed by the tent
// kernel).  The degree used is the smallest p whose prediction is below
// log(eta_tol); a tent whose realised indicator exceeds eta_tol is solved
// again by the tent kernel one degree higher, step by step up to p_max, where
// it is accepted.
//
// Parameter vector (kNParam floats / BF16 values):
//   W1[kHid][kFeat], b1[kHid], W2[kHid][kHid], b2[kHid], W3[kOut][kHid], b3[kOut]
// Activation: tanh.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tdg_internal.h"

namespace tdg {

namespace {

constexpr int oW1 = 0;
constexpr int ob1 = oW1 + kHid * kFeat;
constexpr int oW2 = ob1 + kHid;
constexpr int ob2 = oW2 + kHid * kHid;
constexpr int oW3 = ob2 + kHid;
constexpr int ob3 = oW3 + kOut * kHid;
static_assert(ob3 + kOut == kNParam, "parameter layout");

__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// round to nearest even
__device__ inline unsigned short f32_to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// forward of one sample; w: FP32 copy of the BF16 weights (LDS); x, a1, a2, y:
// this sample's rows (LDS)
__device__ inline void mlp_forward_one(const float* w, const float* x, float* a1, float* a2, float* y) {
  for (int i = 0; i < kHid; ++i) {
    float s = w[ob1 + i];
    for (int k = 0; k < kFeat; ++k) s += w[oW1 + i * kFeat + k] * x[k];
    a1[i] = tanhf(s);
  }
  for (int i = 0; i < kHid; ++i) {
    float s = w[ob2 + i];
    for (int k = 0; k < kHid; ++k) s += w[oW2 + i * kHid + k] * a1[k];
    a2[i] = tanhf(s);
  }
  for (int o = 0; o < kOut; ++o) {
    float s = w[ob3 + o];
    for (int k = 0; k < kHid; ++k) s += w[oW3 + o * kHid + k] * a2[k];
    y[o] = s;
  }
}

__device__ inline void stage_weights(const unsigned short* wb, float* w) {
  for (int i = threadIdx.x; i < kNParam; i += blockDim.x) w[i] = bf16_to_f32(wb[i]);
  __syncthreads();
}

constexpr int kMB = 64;   // samples per block in the forward and selection kernels
constexpr int kMBB = 32;  // samples per block in the backward kernel

__global__ __launch_bounds__(kMB) void mlp_forward_kernel(const unsigned short* wb, const float* x, long long n,
                                                          float* y) {
  __shared__ float w[kNParam];
  __shared__ float sx[kMB][kFeat], sa1[kMB][kHid], sa2[kMB][kHid], sy[kMB][kOut];
  stage_weights(wb, w);
  const int tid = threadIdx.x;
  const long long s = (long long)blockIdx.x * kMB + tid;
  if (s >= n) return;
  for (int k = 0; k < kFeat; ++k) sx[tid][k] = x[s * kFeat + k];
  mlp_forward_one(w, sx[tid], sa1[tid], sa2[tid], sy[tid]);
  for (int o = 0; o < kOut; ++o) y[s * kOut + o] = sy[tid][o];
}

// Per-block gradient of sum_s sum_o mask (y - t)^2 / norm over the block's
// samples; partial[block][kNParam + 1] (last entry: the block's loss sum).
__global__ __launch_bounds__(kMBB) void mlp_backward_kernel(const unsigned short* wb, const float* x, const float* t,
                                                            const float* mask, long long n, float norm,
                                                            float* partial) {
  __shared__ float w[kNParam];
  __shared__ float sx[kMBB][kFeat], sa1[kMBB][kHid], sd1[kMBB][kHid], sa2[kMBB][kHid], sd2[kMBB][kHid];
  __shared__ float sy[kMBB][kOut], sd3[kMBB][kOut];
  __shared__ float sl[kMBB];
  stage_weights(wb, w);
  const int tid = threadIdx.x;
  const long long s = (long long)blockIdx.x * kMBB + tid;
  float loss = 0.0f;
  if (s < n) {
    for (int k = 0; k < kFeat; ++k) sx[tid][k] = x[s * kFeat + k];
    mlp_forward_one(w, sx[tid], sa1[tid], sa2[tid], sy[tid]);
    for (int o = 0; o < kOut; ++o) {
      const float m = mask[s * kOut + o];
      const float r = sy[tid][o] - t[s * kOut + o];
      loss += m * r * r;
      sd3[tid][o] = 2.0f * m * r / norm;
    }
    for (int k = 0; k < kHid; ++k) {
      float g = 0.0f;
      for (int o = 0; o < kOut; ++o) g += w[oW3 + o * kHid + k] * sd3[tid][o];
      sd2[tid][k] = g * (1.0f - sa2[tid][k] * sa2[tid][k]);
    }
    for (int k = 0; k < kHid; ++k) {
      float g = 0.0f;
      for (int i = 0; i < kHid; ++i) g += w[oW2 + i * kHid + k] * sd2[tid][i];
      sd1[tid][k] = g * (1.0f - sa1[tid][k] * sa1[tid][k]);
    }
  } else {
    for (int k = 0; k < kHid; ++k) sd1[tid][k] = sa1[tid][k] = sa2[tid][k] = sd2[tid][k] = 0.0f;
    for (int k = 0; k < kFeat; ++k) sx[tid][k] = 0.0f;
    for (int o = 0; o < kOut; ++o) sd3[tid][o] = 0.0f;
  }
  sl[tid] = loss;
  __syncthreads();
  float* out = partial + (long long)blockIdx.x * (kNParam + 1);
  constexpr int kMB = kMBB;
  for (int pi = tid; pi < kNParam; pi += blockDim.x) {
    float g = 0.0f;
    if (pi < ob1) {
      const int i = (pi - oW1) / kFeat, k = (pi - oW1) % kFeat;
      for (int q = 0; q < kMB; ++q) g += sd1[q][i] * sx[q][k];
    } else if (pi < oW2) {
      const int i = pi - ob1;
      for (int q = 0; q < kMB; ++q) g += sd1[q][i];
    } else if (pi < ob2) {
      const int i = (pi - oW2) / kHid, k = (pi - oW2) % kHid;
      for (int q = 0; q < kMB; ++q) g += sd2[q][i] * sa1[q][k];
    } else if (pi < oW3) {
      const int i = pi - ob2;
      for (int q = 0; q < kMB; ++q) g += sd2[q][i];
    } else if (pi < ob3) {
      const int o = (pi - oW3) / kHid, k = (pi - oW3) % kHid;
      for (int q = 0; q < kMB; ++q) g += sd3[q][o] * sa2[q][k];
    } else {
      const int o = pi - ob3;
      for (int q = 0; q < kMB; ++q) g += sd3[q][o];
    }
    out[pi] = g;
  }
  if (tid == 0) {
    float ls = 0.0f;
    for (int q = 0; q < kMB; ++q) ls += sl[q];
    out[kNParam] = ls / norm;
  }
}

// grad[i] = sum over blocks of partial[b][i] in block order (i = kNParam: loss)
__global__ void mlp_reduce_kernel(const float* partial, int nblocks, float* grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kNParam) return;
  float g = 0.0f;
  for (int b = 0; b < nblocks; ++b) g += partial[(long long)b * (kNParam + 1) + i];
  grad[i] = g;
}

// Fixed scratch of tdg_mlp_backward_noalloc: the per-block partial gradients of
// at most kNoAllocMaxSamples samples.  Each GPU the library runs on holds its
// own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr long long kNoAllocMaxBlocks = kNoAllocMaxSamples / kMBB;
static_assert(kNoAllocMaxSamples % kMBB == 0, "whole blocks");
__device__ __align__(256) float scratch[kNoAllocMaxBlocks * (kNParam + 1)];

__global__ void mlp_adam_kernel(float* w32, unsigned short* wb, const float* grad, float* m, float* v, int step, float lr,
                                float b1, float b2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNParam) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)step));
  const float vh = vi / (1.0f - powf(b2, (float)step));
  const float wn = w32[i] - lr * mh / (sqrtf(vh) + eps);
  w32[i] = wn;
  wb[i] = f32_to_bf16(wn);
}

__global__ void mlp_round_kernel(const float* w32, unsigned short* wb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = f32_to_bf16(w32[i]);
}

// Features of the tents t0 .. t0+count-1 before they are solved (one wave per tent):
//  0 log(dt c_max / h_V)   1 log h_V   2 |patch| / 16   3 log c_max   4 log(c_max / c_min)
//  5 log(E_bot(u_b) / |patch|)  6 log(relative spread of u_b inside the elements)
//  7 1 if V has Dirichlet facets
// h_V = largest distance from X_V to a patch vertex; E_bot as in the tent kernel.
template <int NS>
__global__ __launch_bounds__(64) void tent_features_kernel(KParams P, int t0, int count, float* feats) {
  const int ti = blockIdx.x;
  if (ti >= count) return;
  const int tent = t0 + ti;
  const int lane = threadIdx.x;
  const int V = P.tent_V[tent];
  const double dt = P.tent_tt[tent] - P.tent_tb[tent];
  const int pb = P.v2e_ptr[V], np = P.v2e_ptr[V + 1] - pb;
  const int Q = P.Q;
  double cmax = 0.0, cmin = 1e300, hv = 0.0, area = 0.0, E = 0.0, spread = 0.0, norm = 0.0;
  for (int i = 0; i < np; ++i) {
    const int e = P.v2e[pb + i];
    const int* vs = P.elems + (size_t)e * (NS + 1);
    const double* gl = P.grad_lam + (size_t)e * (NS + 1) * NS;
    const double c = P.c[e];
    cmax = fmax(cmax, c);
    cmin = fmin(cmin, c);
    double g[NS];
    for (int d = 0; d < NS; ++d) g[d] = 0.0;
    for (int k = 0; k <= NS; ++k) {
      const int w = vs[k];
      const double tk = P.tau[w];
      double r2 = 0.0;
      for (int d = 0; d < NS; ++d) {
        const double dx = P.coords[(size_t)w * NS + d] - P.coords[(size_t)V * NS + d];
        r2 += dx * dx;
        g[d] += tk * gl[k * NS + d];
      }
      hv = fmax(hv, sqrt(r2));
    }
    const double* st = P.state + (size_t)e * (NS + 2) * Q;
    // element means of (v/c, sigma)
    double mean[NS + 1], wsum = 0.0;
    for (int d = 0; d <= NS; ++d) mean[d] = 0.0;
    double El = 0.0;
    for (int q = lane; q < Q; q += 64) {
      const double w = P.w_ref[q] * P.absdet[e];
      const double v = st[q];
      double s2 = 0.0, sg = 0.0;
      for (int d = 0; d < NS; ++d) {
        const double sd = st[(1 + d) * Q + q];
        s2 += sd * sd;
        sg += sd * g[d];
        mean[1 + d] += w * sd;
      }
      mean[0] += w * v / c;
      wsum += w;
      El += 0.5 * w * (v * v / (c * c) + s2 - 2.0 * v * sg);
    }
    for (int off = 32; off > 0; off >>= 1) {
      El += __shfl_xor(El, off, 64);
      wsum += __shfl_xor(wsum, off, 64);
      for (int d = 0; d <= NS; ++d) mean[d] += __shfl_xor(mean[d], off, 64);
    }
    for (int d = 0; d <= NS; ++d) mean[d] /= wsum;
    double sp = 0.0, nm = 0.0;
    for (int q = lane; q < Q; q += 64) {
      const double w = P.w_ref[q] * P.absdet[e];
      const double u0 = st[q] / c - mean[0];
      sp += w * u0 * u0;
      nm += w * (st[q] / c) * (st[q] / c);
      for (int d = 0; d < NS; ++d) {
        const double sd = st[(1 + d) * Q + q];
        sp += w * (sd - mean[1 + d]) * (sd - mean[1 + d]);
        nm += w * sd * sd;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      sp += __shfl_xor(sp, off, 64);
      nm += __shfl_xor(nm, off, 64);
    }
    E += El;
    spread += sp;
    norm += nm;
    area += wsum;
  }
  if (lane == 0) {
    float* f = feats + (long long)tent * kFeat;
    f[0] = (float)log(dt * cmax / hv);
    f[1] = (float)log(hv);
    f[2] = (float)(np / 16.0);
    f[3] = (float)log(cmax);
    f[4] = (float)log(cmax / cmin);
    f[5] = (float)log(fmax(E, 0.0) / area + 1e-300);
    f[6] = (float)log(spread / (norm + 1e-300) + 1e-30);
    f[7] = (P.vb_ptr[V + 1] > P.vb_ptr[V]) ? 1.0f : 0.0f;
  }
}

// degree of each tent t0 .. t0+count-1: smallest p in [2, pmax] whose predicted
// log indicator is at most log_tol, else pmax
__global__ __launch_bounds__(kMB) void select_degree_kernel(const unsigned short* wb, const float* feats, int t0,
                                                            int count, float log_tol, int pmax, signed char* p_sel) {
  __shared__ float w[kNParam];
  __shared__ float sx[kMB][kFeat], sa1[kMB][kHid], sa2[kMB][kHid], sy[kMB][kOut];
  stage_weights(wb, w);
  const int tid = threadIdx.x;
  const int i = blockIdx.x * kMB + tid;
  if (i >= count) return;
  const int tent = t0 + i;
  for (int k = 0; k < kFeat; ++k) sx[tid][k] = feats[(long long)tent * kFeat + k];
  float* y = sy[tid];
  mlp_forward_one(w, sx[tid], sa1[tid], sa2[tid], y);
  int p = pmax;
  for (int o = 0; o < kOut && o + 2 <= pmax; ++o)
    if (y[o] <= log_tol) {
      p = o + 2;
      break;
    }
  p_sel[tent] = (signed char)p;
}

}  // namespace

// The queue order of one layer: its tents by chosen degree, highest first, in
// index order inside a degree (one wave; per degree a pass over the layer in
// blocks of 64 places the matching tents by ballot and prefix count).  The
// costliest tents start first, so the cheap ones fill the layer's tail.
__global__ __launch_bounds__(64) void order_by_degree_kernel(const signed char* p_sel, int t0, int count, int pmax,
                                                            int* order) {
  const int lane = threadIdx.x;
  int pos = 0;
  for (int d = pmax; d >= 0; --d) {
    for (int b = 0; b < count; b += 64) {
      const int i = b + lane;
      const int pi = i < count ? (int)p_sel[t0 + i] : 0;
      // (degree 0 collects everything outside 1..pmax: the order is always a permutation)
      const bool hit = i < count && (d == 0 ? (pi <= 0 || pi > pmax) : pi == d);
      const unsigned long long m = __ballot(hit);
      const int before = __popcll(m & ((1ull << lane) - 1ull));
      if (hit) order[t0 + pos + before] = t0 + i;
      pos += __popcll(m);
    }
  }
}

int launch_features(const KParams& P, int t0, int count, float* feats, void* stream) {
  if (count <= 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  if (P.n == 1)
    hipLaunchKernelGGL(tent_features_kernel<1>, dim3(count), dim3(64), 0, s, P, t0, count, feats);
  else if (P.n == 2)
    hipLaunchKernelGGL(tent_features_kernel<2>, dim3(count), dim3(64), 0, s, P, t0, count, feats);
  else
    hipLaunchKernelGGL(tent_features_kernel<3>, dim3(count), dim3(64), 0, s, P, t0, count, feats);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_order(const signed char* p_sel, int t0, int count, int pmax, int* order, void* stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(order_by_degree_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, p_sel, t0, count, pmax, order);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_select(const unsigned short* wb, const float* feats, int t0, int count, float log_tol, int pmax,
                  signed char* p_sel, void* stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(select_degree_kernel, dim3((count + kMB - 1) / kMB), dim3(kMB), 0, (hipStream_t)stream, wb,
                     feats, t0, count, log_tol, pmax, p_sel);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept; each GPU holds its own copy at its own
// address.  The array's name is only a host-side stand-in and is never passed
// to a kernel or a copy.
int noalloc_scratch(float** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static float* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error(std::string("tdg_mlp_backward_noalloc: no usable current device: ") + hipGetErrorString(e));
    return TDG_EHIP;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("tdg_mlp_backward_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
      return TDG_EHIP;
    }
    addr[dev] = static_cast<float*>(p);
  }
  *out = addr[dev];
  return TDG_OK;
}

}  // namespace tdg

// ---- C-ABI of the degree network ----------------------------------------------------
extern "C" {

int tdg_mlp_nparam(void) { return tdg::kNParam; }

int tdg_mlp_forward(const uint16_t* w_bf16, const float* x, int64_t n, float* y, tdg_stream stream) {
  if (!w_bf16 || !x || !y || n < 0) {
    tdg::set_error("tdg_mlp_forward: NULL pointer or n < 0");
    return TDG_EINVAL;
  }
  if (n == 0) return TDG_OK;
  const long long nb = (n + tdg::kMB - 1) / tdg::kMB;
  hipLaunchKernelGGL(tdg::mlp_forward_kernel, dim3((unsigned)nb), dim3(tdg::kMB), 0, (hipStream_t)stream,
                     (const unsigned short*)w_bf16, x, (long long)n, y);
  return hipGetLastError() == hipSuccess ? TDG_OK : TDG_EHIP;
}

int tdg_mlp_backward(const uint16_t* w_bf16, const float* x, const float* target, const float* mask, int64_t n,
                     float norm, float* partial, float* grad, tdg_stream stream) {
  if (!w_bf16 || !x || !target || !mask || !partial || !grad || n <= 0 || !(norm > 0)) {
    tdg::set_error("tdg_mlp_backward: NULL pointer, n < 1 or norm <= 0");
    return TDG_EINVAL;
  }
  const long long nb = (n + tdg::kMBB - 1) / tdg::kMBB;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(tdg::mlp_backward_kernel, dim3((unsigned)nb), dim3(tdg::kMBB), 0, s,
                     (const unsigned short*)w_bf16, x, target, mask, (long long)n, norm, partial);
  hipLaunchKernelGGL(tdg::mlp_reduce_kernel, dim3((tdg::kNParam + 1 + 255) / 256), dim3(256), 0, s, partial, (int)nb,
                     grad);
  return hipGetLastError() == hipSuccess ? TDG_OK : TDG_EHIP;
}

int tdg_mlp_backward_noalloc(const uint16_t* w_bf16, const float* x, const float* target, const float* mask,
                             int64_t n, float norm, float* grad, tdg_stream stream) {
  if (!w_bf16 || !x || !target || !mask || !grad || n <= 0 || !(norm > 0)) {
    tdg::set_error("tdg_mlp_backward_noalloc: NULL pointer, n < 1 or norm <= 0");
    return TDG_EINVAL;
  }
  if (n > tdg::kNoAllocMaxSamples) {
    tdg::set_error("tdg_mlp_backward_noalloc: n = " + std::to_string((long long)n) + " exceeds the fixed scratch (" +
                   std::to_string(tdg::kNoAllocMaxSamples) + " samples)");
    return TDG_EINVAL;
  }
  float* partial = nullptr;
  const int rc = tdg::noalloc_scratch(&partial);
  if (rc != TDG_OK) return rc;
  // every block writes its whole row of partial (kNParam + 1 floats) and the
  // reduction reads only the rows of this call, so nothing needs clearing
  const long long nb = (n + tdg::kMBB - 1) / tdg::kMBB;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(tdg::mlp_backward_kernel, dim3((unsigned)nb), dim3(tdg::kMBB), 0, s,
                     (const unsigned short*)w_bf16, x, target, mask, (long long)n, norm, partial);
  hipLaunchKernelGGL(tdg::mlp_reduce_kernel, dim3((tdg::kNParam + 1 + 255) / 256), dim3(256), 0, s, partial, (int)nb,
                     grad);
  return hipGetLastError() == hipSuccess ? TDG_OK : TDG_EHIP;
}

int tdg_mlp_adam(float* w32, uint16_t* w_bf16, const float* grad, float* m, float* v, int32_t step, float lr, float b1,
                 float b2, float eps, tdg_stream stream) {
  if (!w32 || !w_bf16 || !grad || !m || !v || step < 1) {
    tdg::set_error("tdg_mlp_adam: NULL pointer or step < 1");
    return TDG_EINVAL;
  }
  hipLaunchKernelGGL(tdg::mlp_adam_kernel, dim3((tdg::kNParam + 255) / 256), dim3(256), 0, (hipStream_t)stream, w32,
                     (unsigned short*)w_bf16, grad, m, v, (int)step, lr, b1, b2, eps);
  return hipGetLastError() == hipSuccess ? TDG_OK : TDG_EHIP;
}

int tdg_mlp_round(const float* w32, uint16_t* w_bf16, tdg_stream stream) {
  if (!w32 || !w_bf16) {
    tdg::set_error("tdg_mlp_round: NULL pointer");
    return TDG_EINVAL;
  }
  hipLaunchKernelGGL(tdg::mlp_round_kernel, dim3((tdg::kNParam + 255) / 256), dim3(256), 0, (hipStream_t)stream, w32,
                     (unsigned short*)w_bf16, (int)tdg::kNParam);
  return hipGetLastError() == hipSuccess ? TDG_OK : TDG_EHIP;
}

}  // extern "C"
