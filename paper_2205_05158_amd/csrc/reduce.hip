// NMSE against the linear-gain target (Sec. II-B): E = sum|y - Gx|^2, R = sum|Gx|^2,
// and the count of samples whose |y - Gx|^2 or |Gx|^2 is not finite.  Per-tile
// partials (one workgroup per tile, fixed tree) and a single-workgroup final pass
// that sums each stream's tiles in a fixed order with Neumaier compensation, so
// results are deterministic and accurate in float32.  Also the memoryless ideal
// linear-clipping PA, whose cascade pass is an NMSE tile pass that also writes y and g_u.
#include "kernels.hpp"

namespace dpdmi {

namespace {

constexpr int kRedThreads = 256;
constexpr int kMseTile = 4096;   // values per symbol-MSE tile

// Two compensated sums over the NT threads of the workgroup (fixed tree); every thread
// gets both totals.  sh: 4 * NT floats.
template <int NT = kRedThreads>
__device__ void block_reduce2(Comp& a, Comp& b, float* sh) {
  int t = threadIdx.x;
  sh[t] = a.s; sh[NT + t] = a.c;
  sh[2 * NT + t] = b.s; sh[3 * NT + t] = b.c;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (t < w) {
      Comp x{sh[t], sh[NT + t]}, y{sh[2 * NT + t], sh[3 * NT + t]};
      x.add(sh[t + w]); x.add(sh[NT + t + w]);
      y.add(sh[2 * NT + t + w]); y.add(sh[3 * NT + t + w]);
      sh[t] = x.s; sh[NT + t] = x.c;
      sh[2 * NT + t] = y.s; sh[3 * NT + t] = y.c;
    }
    __syncthreads();
  }
  a = Comp{sh[0], sh[NT]};
  b = Comp{sh[2 * NT], sh[3 * NT]};
  __syncthreads();
}

// Sum of one unsigned count per thread (fixed tree); every thread gets the total.
template <int NT = kRedThreads>
__device__ uint32_t block_sum_u32(uint32_t v, uint32_t* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const uint32_t r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kRedThreads) void k_nmse_tiles(StreamTable st, const float* __restrict__ y,
                                                            const float* __restrict__ x, float g_re,
                                                            float g_im, float4* __restrict__ part) {
  __shared__ float sh[4 * kRedThreads];
  __shared__ uint32_t shn[kRedThreads];
  int t = blockIdx.x;
  int s = stream_of_tile(st, t);
  int64_t lo = st.off[s], hi = st.off[s + 1];
  int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * st.tile;
  int64_t t1 = min(hi, t0 + st.tile);
  Comp E, R;
  uint32_t nf = 0;
  for (int64_t n = t0 + threadIdx.x; n < t1; n += kRedThreads) {
    float2 yv = ld2(y, n), xv = ld2(x, n);
    float tr = g_re * xv.x - g_im * xv.y, ti = g_re * xv.y + g_im * xv.x;
    float er = yv.x - tr, ei = yv.y - ti;
    const float e2 = er * er + ei * ei, r2 = tr * tr + ti * ti;
    nf += !isfinite(e2 + r2);
    E.add(e2);
    R.add(r2);
  }
  block_reduce2(E, R, sh);
  nf = block_sum_u32(nf, shn);
  if (threadIdx.x == 0) part[t] = make_float4(E.value(), R.value(), (float)nf, 0.f);
}

// First stage of the final pass: workgroup b sums the tile partials of chunk b (up to
// kNmseChunk consecutive tiles of one stream; chunks never cross streams) in a fixed tree
// into one (E, R, non-finite count) record.  ct: the chunk table (ct.tile0[s] = first
// chunk of stream s).
__global__ __launch_bounds__(kRedThreads) void k_nmse_chunks(StreamTable st, StreamTable ct,
                                                             const float4* __restrict__ part,
                                                             float4* __restrict__ chunk_part) {
  static_assert(kNmseChunk == kRedThreads, "one tile partial per thread");
  __shared__ float sh[4 * kRedThreads];
  __shared__ uint32_t shn[kRedThreads];
  const int b = blockIdx.x;
  const int s = stream_of_tile(ct, b);
  const int t = st.tile0[s] + (b - ct.tile0[s]) * kNmseChunk + (int)threadIdx.x;
  Comp E, R;
  uint32_t nf = 0;
  if (t < st.tile0[s + 1]) {
    const float4 v = part[t];
    E.add(v.x);
    R.add(v.y);
    nf = (uint32_t)v.z;
  }
  block_reduce2(E, R, sh);
  nf = block_sum_u32(nf, shn);
  if (threadIdx.x == 0) chunk_part[b] = make_float4(E.value(), R.value(), (float)nf, 0.f);
}

// Records of DPD_NMSE_FIELDS floats: (E, R, NMSE dB, non-finite count), from the chunk
// records of the first stage (part, indexed by the chunk table st).
constexpr int kFinThreads = 1024;
constexpr int kFinWaves = kFinThreads / 64;

// Sum of a compensated value over the 64 lanes of a wave (fixed butterfly order); lane 0
// holds the result.
__device__ __forceinline__ Comp wave_sum(Comp v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float os = __shfl_xor(v.s, off), oc = __shfl_xor(v.c, off);
    v.add(os);
    v.add(oc);
  }
  return v;
}

// One wave per stream (streams wave, wave + kFinWaves, ...): each lane sums its chunk
// records in stride order, the wave combines them; then thread 0 writes the records and
// pools the streams in stream order.
__global__ __launch_bounds__(kFinThreads) void k_nmse_final(StreamTable st, const float4* __restrict__ part,
                                                            float* __restrict__ rec,
                                                            float* __restrict__ loss,
                                                            float* __restrict__ inv_r) {
  constexpr int F = DPD_NMSE_FIELDS;
  __shared__ float4 sums[DPD_MAX_STREAMS];       // E.s, E.c, R.s, R.c per stream
  __shared__ uint32_t counts[DPD_MAX_STREAMS];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int s = wave; s < st.n; s += kFinWaves) {
    Comp E, R;
    uint32_t nf = 0;
    for (int t = st.tile0[s] + lane; t < st.tile0[s + 1]; t += 64) {
      const float4 v = part[t];
      E.add(v.x);
      R.add(v.y);
      nf += (uint32_t)v.z;
    }
    E = wave_sum(E);
    R = wave_sum(R);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nf += __shfl_xor(nf, off);
    if (lane == 0) {
      sums[s] = make_float4(E.s, E.c, R.s, R.c);
      counts[s] = nf;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Comp Et, Rt;   // pooled over all streams
    uint32_t nft = 0;
    for (int s = 0; s < st.n; ++s) {
      const float4 v = sums[s];
      const Comp E{v.x, v.y}, R{v.z, v.w};
      const float e = E.value(), r = R.value();
      if (rec) {
        rec[F * s] = e;
        rec[F * s + 1] = r;
        rec[F * s + 2] = 10.f * log10f(e / r);
        rec[F * s + 3] = (float)counts[s];
      }
      nft += counts[s];
      Et.add(E.s); Et.add(E.c);
      Rt.add(R.s); Rt.add(R.c);
      if (st.per_stream) {
        if (loss) loss[s] = e / r;
        if (inv_r) inv_r[s] = 1.f / r;
      }
    }
    const float e = Et.value(), r = Rt.value();
    if (rec) {
      rec[F * st.n] = e;
      rec[F * st.n + 1] = r;
      rec[F * st.n + 2] = 10.f * log10f(e / r);
      rec[F * st.n + 3] = (float)nft;
    }
    if (!st.per_stream) {
      if (loss) loss[0] = e / r;
      if (inv_r) inv_r[0] = 1.f / r;
    }
  }
}

// Symbol MSE: per tile of kMseTile values the compensated sum of |z - t|^2 and the
// count of non-finite terms, and (when grad is not null) grad = scale (z - t).
__global__ __launch_bounds__(kRedThreads) void k_mse_tiles(int64_t n, const float* __restrict__ z,
                                                           const float* __restrict__ tg, float scale,
                                                           float* __restrict__ grad,
                                                           float4* __restrict__ part) {
  __shared__ float sh[4 * kRedThreads];
  __shared__ uint32_t shn[kRedThreads];
  const int64_t t0 = (int64_t)blockIdx.x * kMseTile;
  const int64_t t1 = min(n, t0 + kMseTile);
  Comp E, dummy;
  uint32_t nf = 0;
  for (int64_t i = t0 + threadIdx.x; i < t1; i += kRedThreads) {
    const float2 zv = ld2(z, i), tv = ld2(tg, i);
    const float er = zv.x - tv.x, ei = zv.y - tv.y;
    const float e2 = er * er + ei * ei;
    nf += !isfinite(e2);
    E.add(e2);
    if (grad) st2(grad, i, make_float2(scale * er, scale * ei));
  }
  block_reduce2(E, dummy, sh);
  nf = block_sum_u32(nf, shn);
  if (threadIdx.x == 0) part[blockIdx.x] = make_float4(E.value(), 0.f, (float)nf, 0.f);
}

// out[0] = (sum over the tiles, fixed order) / n, out[1] = non-finite count.
__global__ __launch_bounds__(kRedThreads) void k_mse_final(int n_tiles, int64_t n,
                                                           const float4* __restrict__ part,
                                                           float* __restrict__ out) {
  __shared__ float sh[4 * kRedThreads];
  __shared__ uint32_t shn[kRedThreads];
  Comp E, dummy;
  uint32_t nf = 0;
  for (int t = threadIdx.x; t < n_tiles; t += kRedThreads) {
    const float4 v = part[t];
    E.add(v.x);
    nf += (uint32_t)v.z;
  }
  block_reduce2(E, dummy, sh);
  nf = block_sum_u32(nf, shn);
  if (threadIdx.x == 0) {
    out[0] = (float)((double)E.value() / (double)n);
    out[1] = (float)nf;
  }
}

// ------------------------------------------------------------------ linear-clipping PA
// The ideal linear-clipping PA of the paper's SER comparison (Sec. V-B-2): unit gain up
// to the clipping level a, constant envelope a beyond it, phase kept:
//   y = u if |u| <= a,   y = (a / |u|) u otherwise.
// |u| without overflow for every finite u (the square is rescaled when it overflows);
// a NaN sample takes the linear branch and stays NaN.
__device__ __forceinline__ float clip_mag(float2 u) {
  const float r2 = u.x * u.x + u.y * u.y;
  if (r2 != INFINITY) return sqrtf(r2);                 // finite, or NaN
  const float m = fmaxf(fabsf(u.x), fabsf(u.y));
  if (m == INFINITY) return INFINITY;
  const float p = u.x / m, q = u.y / m;
  return m * sqrtf(p * p + q * q);
}

__global__ __launch_bounds__(kRedThreads) void k_clip_fwd(int64_t n, const float* __restrict__ u, float a,
                                                          float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    float2 v = ld2(u, i);
    const float r = clip_mag(v);
    if (r > a) {
      const float sc = a / r;
      v = make_float2(sc * v.x, sc * v.y);
    }
    st2(y, i, v);
  }
}

// The clipping PA with the NMSE partials and its reverse mode over the table's tiles:
// y (may be null), (E, R, non-finite count) per tile, and (when gu is not null)
// g_u = J^T g_y with g_y = 2 (y - G x) (the loss's 1/R is applied with dW).  J = I on
// the linear branch; beyond the clip J = (a / |u|)(I - v v^T), v = u / |u|: only the
// phase of u moves y.  At |u| = a the linear branch's derivative is taken.
__global__ __launch_bounds__(kRedThreads) void k_clip_tiles(StreamTable st, const float* __restrict__ x,
                                                            const float* __restrict__ u, float a,
                                                            float g_re, float g_im,
                                                            float4* __restrict__ part,
                                                            float* __restrict__ gu,
                                                            float* __restrict__ y) {
  __shared__ float sh[4 * kRedThreads];
  __shared__ uint32_t shn[kRedThreads];
  const int t = blockIdx.x;
  const int s = stream_of_tile(st, t);
  const int64_t lo = st.off[s], hi = st.off[s + 1];
  const int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * st.tile;
  const int64_t t1 = min(hi, t0 + st.tile);
  Comp E, R;
  uint32_t nf = 0;
  for (int64_t n = t0 + threadIdx.x; n < t1; n += kRedThreads) {
    const float2 uv = ld2(u, n), xv = ld2(x, n);
    const float r = clip_mag(uv);
    const bool clipped = r > a;
    const float sc = clipped ? a / r : 1.f;
    const float2 yv = make_float2(sc * uv.x, sc * uv.y);
    const float tr = g_re * xv.x - g_im * xv.y, ti = g_re * xv.y + g_im * xv.x;
    const float er = yv.x - tr, ei = yv.y - ti;
    const float e2 = er * er + ei * ei, r2 = tr * tr + ti * ti;
    nf += !isfinite(e2 + r2);
    E.add(e2);
    R.add(r2);
    if (y) st2(y, n, yv);
    if (gu) {
      float gx = 2.f * er, gy = 2.f * ei;
      if (clipped) {
        const float vx = uv.x / r, vy = uv.y / r;
        const float d = vx * gx + vy * gy;
        gx = sc * (gx - d * vx);
        gy = sc * (gy - d * vy);
      }
      st2(gu, n, make_float2(gx, gy));
    }
  }
  block_reduce2(E, R, sh);
  nf = block_sum_u32(nf, shn);
  if (threadIdx.x == 0) part[t] = make_float4(E.value(), R.value(), (float)nf, 0.f);
}

}  // namespace

void launch_clip_fwd(int64_t n, const float* u, float a, float* y, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(ceil_div64(n, kRedThreads), 8192);
  k_clip_fwd<<<(unsigned)blocks, kRedThreads, 0, s>>>(n, u, a, y);
}

void launch_clip_tiles(const StreamTable& st, const float* x, const float* u, float a, float g_re,
                       float g_im, float4* tile_part, float* gu, float* y, hipStream_t s) {
  k_clip_tiles<<<st.n_tiles, kRedThreads, 0, s>>>(st, x, u, a, g_re, g_im, tile_part, gu, y);
}

int mse_tiles(int64_t n) { return (int)ceil_div64(n, kMseTile); }

void launch_mse(int64_t n, const float* z, const float* t, float scale, float* grad, float4* part,
                float* out, hipStream_t s) {
  const int nt = mse_tiles(n);
  k_mse_tiles<<<nt, kRedThreads, 0, s>>>(n, z, t, scale, grad, part);
  k_mse_final<<<1, kRedThreads, 0, s>>>(nt, n, part, out);
}

void launch_nmse_tiles(const StreamTable& st, const float* y, const float* x, float g_re,
                       float g_im, float4* tile_part, hipStream_t s) {
  k_nmse_tiles<<<st.n_tiles, kRedThreads, 0, s>>>(st, y, x, g_re, g_im, tile_part);
}

StreamTable nmse_chunk_table(const StreamTable& st) {
  StreamTable ct = st;
  ct.tile = st.tile * kNmseChunk;
  int32_t c = 0;
  for (int i = 0; i < st.n; ++i) {
    ct.tile0[i] = c;
    c += (st.tile0[i + 1] - st.tile0[i] + kNmseChunk - 1) / kNmseChunk;
  }
  ct.tile0[st.n] = c;
  ct.n_tiles = c;
  return ct;
}

void launch_nmse_final(const StreamTable& st, float4* tile_part, float* rec, float* loss, float* inv_r,
                       hipStream_t s) {
  const StreamTable ct = nmse_chunk_table(st);
  float4* chunk_part = tile_part + st.n_tiles;
  k_nmse_chunks<<<ct.n_tiles, kRedThreads, 0, s>>>(st, ct, tile_part, chunk_part);
  k_nmse_final<<<1, kFinThreads, 0, s>>>(ct, chunk_part, rec, loss, inv_r);
}

}  // namespace dpdmi
