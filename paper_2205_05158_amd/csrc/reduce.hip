// NMSE against the linear-gain target (Sec. II-B): E = sum|y - Gx|^2, R = sum|Gx|^2.
// Per-tile partials (one workgroup per tile, fixed tree) and a single-workgroup
// final pass that sums each stream's tiles in a fixed order with Neumaier
// compensation, so results are deterministic and accurate in float32.
#include "kernels.hpp"

namespace dpdmi {

namespace {

constexpr int kRedThreads = 256;

__device__ void block_reduce2(Comp& a, Comp& b, float* sh) {
  // sh: 4 * kRedThreads floats
  int t = threadIdx.x;
  sh[t] = a.s; sh[kRedThreads + t] = a.c;
  sh[2 * kRedThreads + t] = b.s; sh[3 * kRedThreads + t] = b.c;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      Comp x{sh[t], sh[kRedThreads + t]}, y{sh[2 * kRedThreads + t], sh[3 * kRedThreads + t]};
      x.add(sh[t + w]); x.add(sh[kRedThreads + t + w]);
      y.add(sh[2 * kRedThreads + t + w]); y.add(sh[3 * kRedThreads + t + w]);
      sh[t] = x.s; sh[kRedThreads + t] = x.c;
      sh[2 * kRedThreads + t] = y.s; sh[3 * kRedThreads + t] = y.c;
    }
    __syncthreads();
  }
  a = Comp{sh[0], sh[kRedThreads]};
  b = Comp{sh[2 * kRedThreads], sh[3 * kRedThreads]};
  __syncthreads();
}

__global__ __launch_bounds__(kRedThreads) void k_nmse_tiles(StreamTable st, const float* __restrict__ y,
                                                            const float* __restrict__ x, float g_re,
                                                            float g_im, float2* __restrict__ part) {
  __shared__ float sh[4 * kRedThreads];
  int t = blockIdx.x;
  int s = stream_of_tile(st, t);
  int64_t lo = st.off[s], hi = st.off[s + 1];
  int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * st.tile;
  int64_t t1 = min(hi, t0 + st.tile);
  Comp E, R;
  for (int64_t n = t0 + threadIdx.x; n < t1; n += kRedThreads) {
    float2 yv = ld2(y, n), xv = ld2(x, n);
    float tr = g_re * xv.x - g_im * xv.y, ti = g_re * xv.y + g_im * xv.x;
    float er = yv.x - tr, ei = yv.y - ti;
    E.add(er * er + ei * ei);
    R.add(tr * tr + ti * ti);
  }
  block_reduce2(E, R, sh);
  if (threadIdx.x == 0) part[t] = make_float2(E.value(), R.value());
}

__global__ __launch_bounds__(kRedThreads) void k_nmse_final(StreamTable st, const float2* __restrict__ part,
                                                            float* __restrict__ out3,
                                                            float* __restrict__ loss,
                                                            float* __restrict__ inv_r) {
  __shared__ float sh[4 * kRedThreads];
  Comp Et, Rt;   // pooled over all streams
  for (int s = 0; s < st.n; ++s) {
    Comp E, R;
    for (int t = st.tile0[s] + threadIdx.x; t < st.tile0[s + 1]; t += kRedThreads) {
      float2 v = part[t];
      E.add(v.x);
      R.add(v.y);
    }
    block_reduce2(E, R, sh);
    float e = E.value(), r = R.value();
    if (threadIdx.x == 0) {
      if (out3) {
        out3[3 * s] = e;
        out3[3 * s + 1] = r;
        out3[3 * s + 2] = 10.f * log10f(e / r);
      }
      Et.add(E.s); Et.add(E.c);
      Rt.add(R.s); Rt.add(R.c);
      if (st.per_stream) {
        if (loss) loss[s] = e / r;
        if (inv_r) inv_r[s] = 1.f / r;
      }
    }
  }
  if (threadIdx.x == 0) {
    float e = Et.value(), r = Rt.value();
    if (out3) {
      out3[3 * st.n] = e;
      out3[3 * st.n + 1] = r;
      out3[3 * st.n + 2] = 10.f * log10f(e / r);
    }
    if (!st.per_stream) {
      if (loss) loss[0] = e / r;
      if (inv_r) inv_r[0] = 1.f / r;
    }
  }
}

}  // namespace

void launch_nmse_tiles(const StreamTable& st, const float* y, const float* x, float g_re,
                       float g_im, float2* tile_part, hipStream_t s) {
  k_nmse_tiles<<<st.n_tiles, kRedThreads, 0, s>>>(st, y, x, g_re, g_im, tile_part);
}

void launch_nmse_final(const StreamTable& st, const float2* tile_part, float* out3, float* loss,
                       float* inv_r, hipStream_t s) {
  k_nmse_final<<<1, kRedThreads, 0, s>>>(st, tile_part, out3, loss, inv_r);
}

}  // namespace dpdmi
