// Adam update of the DPD parameters on the device: the optimiser the paper trains its
// DPD networks with (Sec. V-A-2), with the update rule of the optimiser's own paper
// (Kingma & Ba, Algorithm 1).  Elementwise and HBM-bound (16 bytes read, 12 written per
// parameter): one thread per 4 parameters with 16-byte accesses when the buffers allow,
// grid-stride over the vector.
#include "kernels.hpp"

namespace dpdmi {

namespace {

// Hyper-parameters as float32 operands; 1 - beta is rounded from the double-precision
// value (rounding beta first would cost 1 - 0.999 about 1e-5 relative).
struct AdamArgs {
  float lr, beta1, beta2, eps;
  float omb1, omb2;   // 1 - beta1, 1 - beta2
  float c1, c2;       // 1 / (1 - beta1^t), 1 / (1 - beta2^t)
};

__device__ __forceinline__ void adam_one(float g, float& w, float& m, float& v, const AdamArgs& a) {
  m = fmaf(a.beta1, m, a.omb1 * g);
  v = fmaf(a.beta2, v, a.omb2 * (g * g));
  const float mh = m * a.c1, vh = v * a.c2;
  w -= a.lr * mh / (sqrtf(vh) + a.eps);
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_adam(const float* __restrict__ g, float* __restrict__ w,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n,
                                              AdamArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (VEC) {
    const int64_t n4 = n / 4;
    for (int64_t i = i0; i < n4; i += stride) {
      const float4 gv = reinterpret_cast<const float4*>(g)[i];
      float4 wv = reinterpret_cast<float4*>(w)[i];
      float4 mv = reinterpret_cast<float4*>(m)[i];
      float4 vv = reinterpret_cast<float4*>(v)[i];
      adam_one(gv.x, wv.x, mv.x, vv.x, a);
      adam_one(gv.y, wv.y, mv.y, vv.y, a);
      adam_one(gv.z, wv.z, mv.z, vv.z, a);
      adam_one(gv.w, wv.w, mv.w, vv.w, a);
      reinterpret_cast<float4*>(w)[i] = wv;
      reinterpret_cast<float4*>(m)[i] = mv;
      reinterpret_cast<float4*>(v)[i] = vv;
    }
    for (int64_t i = 4 * n4 + i0; i < n; i += stride) adam_one(g[i], w[i], m[i], v[i], a);
  } else {
    for (int64_t i = i0; i < n; i += stride) adam_one(g[i], w[i], m[i], v[i], a);
  }
}

}  // namespace

void launch_adam(const float* g, float* w, float* m, float* v, int64_t n, int step, double lr,
                 double beta1, double beta2, double eps, int cus, hipStream_t s) {
  AdamArgs a;
  a.lr = (float)lr;
  a.beta1 = (float)beta1;
  a.beta2 = (float)beta2;
  a.eps = (float)eps;
  a.omb1 = (float)(1.0 - beta1);
  a.omb2 = (float)(1.0 - beta2);
  a.c1 = (float)(1.0 / (1.0 - pow(beta1, (double)step)));
  a.c2 = (float)(1.0 / (1.0 - pow(beta2, (double)step)));
  const bool vec = ((uintptr_t)g | (uintptr_t)w | (uintptr_t)m | (uintptr_t)v) % 16 == 0;
  const int64_t work = vec ? (n + 3) / 4 : n;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 8 * (int64_t)cus));
  if (vec) k_adam<true><<<grid, 256, 0, s>>>(g, w, m, v, n, a);
  else k_adam<false><<<grid, 256, 0, s>>>(g, w, m, v, n, a);
}

}  // namespace dpdmi
