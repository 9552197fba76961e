// Least-squares identification of a GMP DPD by indirect learning: the TD-GMP benchmark
// of the paper (the per-antenna DPD of eq. (9), coefficients by mean-square-error
// estimation, Sec. III-B) fitted as a post-inverse at the PA output (Sec. V-A-2).
//
// The normal equations Phi^H Phi c = Phi^H t are accumulated on the FP64 matrix cores
// (the basis is badly conditioned: powers |z|^k of one envelope; float32 sums would not
// survive the solve), then solved per parameter set by a complex Cholesky factorisation
// in one workgroup.
//
// Real embedding: with Phi = A + iB and t = t_r + i t_i, the matrix P = [A B t_r t_i]
// (N x NC, NC = 2J + 2, padded to NCP, a multiple of 64) has the symmetric Gram
// Q = P^T P, from which
//   Phi^H Phi = (A^T A + B^T B) + i (A^T B - B^T A),
//   Phi^H t   = (A^T t_r + B^T t_i) + i (A^T t_i - B^T t_r).
// Q is computed in 128 x 128 blocks of its upper block triangle (the last block row and
// column are 64 wide when NCP is an odd multiple of 64; the waves whose tiles fall past
// them skip their MFMAs); each workgroup (8 waves,
// each 2 x 4 tiles of 16 x 16) owns one block and a contiguous range of 32-sample chunks,
// builds the basis values of its block's row and column sets (one set on the diagonal)
// for each chunk in LDS (from the stream's z window and |z|^k table) and runs 16x16x4 f64
// MFMAs (8 per basis value built off the diagonal); partial blocks go to one slot per
// (sample split, stream), summed in a fixed order by k_ls_reduce.
#include "kernels.hpp"

namespace dpdmi {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kLsThreads = 512;     // 8 waves
constexpr int kLsChunk = 16;        // samples per basis chunk (4 MFMA K steps)
constexpr int kLsBlk = kLsGramBlk;  // Gram block edge (128)
// LDS row stride (doubles) of a chunk's basis rows: 144 doubles = 288 banks, 32 mod 64, so
// the two sample rows a 32-lane half of an operand read touches use disjoint banks
constexpr int kLsRow = kLsBlk + 16;
constexpr int kLsMaxWin = kLsChunk + DPD_MAX_GMP_M + 2 * DPD_MAX_GMP_L;

// Column descriptor of the real embedding: kind 0 Re phi_j, 1 Im phi_j, 2 Re t, 3 Im t,
// 4 zero padding; for phi_j the monomial z[n - l] |z[n - q]|^k.
struct ColDesc {
  int kind, k, l, q;
};

__host__ __device__ inline ColDesc col_desc(int c, int K, int M, int L, int J) {
  ColDesc d{4, 0, 0, 0};
  if (c >= 2 * J + 2) return d;
  if (c >= 2 * J) { d.kind = 2 + (c - 2 * J); return d; }
  d.kind = c >= J ? 1 : 0;
  int j = c >= J ? c - J : c;
  const int na = K * (M + 1), nb = (K - 1) * (M + 1) * L;
  if (j < na) {
    d.k = j / (M + 1);
    d.l = j % (M + 1);
    d.q = d.l;
    return d;
  }
  j -= na;
  const int sign = j < nb ? +1 : -1;          // b: lag q = l + g; c: lead q = l - g
  if (j >= nb) j -= nb;
  const int g = j % L + 1;
  d.l = (j / L) % (M + 1);
  d.k = j / (L * (M + 1)) + 1;
  d.q = d.l + sign * g;
  return d;
}

// Block index (upper block triangle, row-major) -> (block row, block col).
__host__ __device__ inline void blk_of(int b, int nb, int& bi, int& bj) {
  bi = 0;
  while (b >= nb - bi) { b -= nb - bi; ++bi; }
  bj = bi + b;
}

struct LsGeom {
  int K, M, L, J, NCP, nb, nblk;
};

__global__ __launch_bounds__(kLsThreads) void k_ls_gram(StreamTable st, LsGeom gm, const float* __restrict__ y,
                                                        double gi_re, double gi_im,
                                                        const float* __restrict__ t, int n_splits,
                                                        double* __restrict__ slots) {
  __shared__ double2 zw[kLsMaxWin];
  __shared__ double rp[DPD_MAX_GMP_K][kLsMaxWin];
  __shared__ double2 tw[kLsChunk];
  __shared__ int4 cd[2 * kLsBlk];
  __shared__ double pb[2][kLsChunk][kLsRow];    // basis rows of the block's row / col columns

  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  int bi, bj;
  blk_of(blockIdx.x, gm.nb, bi, bj);
  const bool diag = bi == bj;                  // row and column sets coincide
  const int tr0 = 2 * (wave % 4), tc0 = 4 * (wave / 4);   // the wave's tile rows / columns
  // the last block row / column may be 64 wide: waves whose tiles lie past it skip the MFMAs
  const bool active = 16 * tr0 < min(kLsBlk, gm.NCP - kLsBlk * bi) && 16 * tc0 < min(kLsBlk, gm.NCP - kLsBlk * bj);
  const int split = blockIdx.y;
  const int t_begin = wg_tile_start(split, n_splits, st.n_tiles);
  const int t_end = wg_tile_start(split + 1, n_splits, st.n_tiles);
  const int HB = gm.M + gm.L;                  // window positions before the chunk
  const int WS = kLsChunk + gm.M + 2 * gm.L;   // z window [n0 - M - L, n0 + chunk + L)
  if (tid < 2 * kLsBlk) {
    const int c = (tid < kLsBlk ? kLsBlk * bi : kLsBlk * bj) + tid % kLsBlk;
    const ColDesc d = col_desc(c, gm.K, gm.M, gm.L, gm.J);
    cd[tid] = make_int4(d.kind, d.k, HB - d.l, HB - d.q);   // window offsets of z[n-l], |z[n-q]|
  }
  f64x4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  auto flush = [&](int s) {
    double* out = slots + ((int64_t)(split + s) * gm.nblk + blockIdx.x) * (kLsBlk * kLsBlk);
    // D layout of 16x16x4 f64: lane l holds column l % 16, rows l / 16 + 4 r
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (tr0 + i) + lane / 16 + 4 * r, col = 16 * (tc0 + j) + lane % 16;
          out[row * kLsBlk + col] = acc[i][j][r];
        }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  };
  // basis build: thread tid owns column tid % ncol of the row set (then the column set)
  // for samples tid / ncol + k * (threads / ncol)
  const int ncol = diag ? kLsBlk : 2 * kLsBlk;
  const int my_c = tid % ncol, s_first = tid / ncol, s_step = kLsThreads / ncol;
  __syncthreads();
  const int4 my_d = cd[my_c];

  // the next chunk's y window and targets are read one chunk ahead, into registers
  // (thread i < WS holds window position i, thread i < chunk target i)
  float2 ypre = make_float2(0.f, 0.f), tpre = make_float2(0.f, 0.f);
  auto prefetch = [&](int tt) {
    const int s2 = stream_of_tile(st, tt);
    const int64_t lo2 = st.off[s2], hi2 = st.off[s2 + 1];
    const int64_t n02 = lo2 + (int64_t)(tt - st.tile0[s2]) * kLsChunk;
    const int64_t p = n02 - HB + tid;
    ypre = (tid < WS && p >= lo2 && p < hi2) ? ld2(y, p) : make_float2(0.f, 0.f);
    tpre = (tid < kLsChunk && n02 + tid < hi2) ? ld2(t, n02 + tid) : make_float2(0.f, 0.f);
  };
  static_assert(kLsMaxWin <= kLsThreads, "one window position per thread");
  if (t_begin < t_end) prefetch(t_begin);

  int cur = -1;
  for (int tt = t_begin; tt < t_end; ++tt) {
    const int s = stream_of_tile(st, tt);
    const int64_t hi = st.off[s + 1];
    const int64_t n0 = st.off[s] + (int64_t)(tt - st.tile0[s]) * kLsChunk;
    if (s != cur) {
      if (cur >= 0) flush(cur);
      cur = s;
    }
    __syncthreads();   // previous chunk's basis consumed
    if (tid < WS) {
      const double2 z = make_double2(ypre.x * gi_re - ypre.y * gi_im, ypre.x * gi_im + ypre.y * gi_re);
      zw[tid] = z;
      const double r = sqrt(z.x * z.x + z.y * z.y);
      double pw = 1.0;
      for (int k = 0; k < gm.K; ++k) {
        rp[k][tid] = pw;
        pw *= r;
      }
    }
    if (tid < kLsChunk) tw[tid] = make_double2(tpre.x, tpre.y);
    if (tt + 1 < t_end) prefetch(tt + 1);
    __syncthreads();
    // basis values of the chunk (rows past the stream are zero)
    double* mycol = &pb[my_c / kLsBlk][0][my_c % kLsBlk];
    for (int smp = s_first; smp < kLsChunk; smp += s_step) {
      double v = 0.0;
      if (n0 + smp < hi) {
        if (my_d.x <= 1) {
          const double2 zl = zw[smp + my_d.z];
          const double rq = rp[my_d.y][smp + my_d.w];
          v = (my_d.x == 0 ? zl.x : zl.y) * rq;
        } else if (my_d.x == 2) {
          v = tw[smp].x;
        } else if (my_d.x == 3) {
          v = tw[smp].y;
        }
      }
      mycol[smp * kLsRow] = v;
    }
    __syncthreads();
    // Q block += P[chunk][rows]^T P[chunk][cols]: A[i][k] = P[4 kk + k][row 16 tr + i] from
    // lane i + 16 k, B[k][j] = P[4 kk + k][col 16 tc + j] from lane j + 16 k
    const double(*pcol)[kLsRow] = pb[diag ? 0 : 1];
    if (!active) continue;
#pragma unroll
    for (int kk = 0; kk < kLsChunk / 4; ++kk) {
      const int smp = 4 * kk + lane / 16;
      const double a0 = pb[0][smp][16 * tr0 + lane % 16];
      const double a1 = pb[0][smp][16 * (tr0 + 1) + lane % 16];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double b = pcol[smp][16 * (tc0 + j) + lane % 16];
        acc[0][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc[0][j], 0, 0, 0);
        acc[1][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc[1][j], 0, 0, 0);
      }
    }
  }
  if (cur >= 0) flush(cur);
}

// Sum of the slots of parameter set `set` (streams of the set in order, splits in order)
// into the complex normal matrix [J][J + 1] (Phi^H Phi | Phi^H t), from the real Gram.
__global__ void k_ls_reduce(StreamTable st, LsGeom gm, int n_splits, const double* __restrict__ slots,
                            double2* __restrict__ normal) {
  const int set = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int J = gm.J;
  if (idx >= (int64_t)J * (J + 1)) return;
  const int i = (int)(idx / (J + 1)), jj = (int)(idx % (J + 1));
  // Q[r][c] from the upper block triangle of one slot
  auto q = [&](const double* sl, int r, int c) {
    int br = r / kLsBlk, bc = c / kLsBlk;
    if (br > bc) { int tmp = r; r = c; c = tmp; tmp = br; br = bc; bc = tmp; }
    const int b = br * gm.nb - br * (br - 1) / 2 + (bc - br);
    return sl[(int64_t)b * (kLsBlk * kLsBlk) + (r % kLsBlk) * kLsBlk + c % kLsBlk];
  };
  double re = 0.0, im = 0.0;
  for (int s = 0; s < st.n; ++s) {
    if ((st.per_stream ? s : 0) != set) continue;
    if (st.tile0[s] == st.tile0[s + 1]) continue;
    const int g0 = wg_of_tile(st.tile0[s], n_splits, st.n_tiles);
    const int g1 = wg_of_tile(st.tile0[s + 1] - 1, n_splits, st.n_tiles);
    for (int g = g0; g <= g1; ++g) {
      const double* sl = slots + (int64_t)(g + s) * gm.nblk * (kLsBlk * kLsBlk);
      if (jj < J) {
        re += q(sl, i, jj) + q(sl, J + i, J + jj);
        im += q(sl, i, J + jj) - q(sl, J + i, jj);
      } else {
        re += q(sl, i, 2 * J) + q(sl, J + i, 2 * J + 1);
        im += q(sl, i, 2 * J + 1) - q(sl, J + i, 2 * J);
      }
    }
  }
  normal[(int64_t)set * J * (J + 1) + idx] = make_double2(re, im);
}

__device__ inline double2 cmul_d(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc_d(double2 a, double2 b) {   // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// One workgroup per parameter set: (H + lambda I) c = rhs with H = normal[:, :J] Hermitian
// positive definite, by a right-looking complex Cholesky factorisation H = L L^H in the
// work copy (lower triangle), then L w = rhs and L^H c = w.  info[set] = 0, or k + 1 when
// pivot k is not positive (c is then left zero).
constexpr int kLsSolveThreads = 512;

__global__ __launch_bounds__(kLsSolveThreads) void k_ls_solve(LsGeom gm, const double2* __restrict__ normal,
                                                  double ridge, double2* __restrict__ work,
                                                  float* __restrict__ coef, int* __restrict__ info) {
  const int set = blockIdx.x, tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int J = gm.J;
  __shared__ double2 lk[kLsMaxJ];
  const double2* Hn = normal + (int64_t)set * J * (J + 1);
  double2* A = work + (int64_t)set * J * (J + 1);          // [J][J], column J = right-hand side
  __shared__ double red[kLsSolveThreads];
  __shared__ double lam;
  __shared__ int bad;
  // ridge: lambda = ridge * tr(H) / J
  double tr = 0.0;
  for (int i = tid; i < J; i += kLsSolveThreads) tr += Hn[(int64_t)i * (J + 1) + i].x;
  red[tid] = tr;
  __syncthreads();
  for (int w = kLsSolveThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) { lam = ridge * red[0] / J; bad = 0; }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)J * (J + 1); e += kLsSolveThreads) {
    double2 v = Hn[e];
    const int r = (int)(e / (J + 1)), c = (int)(e % (J + 1));
    if (r == c) v.x += lam;
    A[e] = v;
  }
  __syncthreads();
  const int ld = J + 1;
  for (int k = 0; k < J; ++k) {
    if (tid == 0) {
      const double d = A[(int64_t)k * ld + k].x;
      if (!(d > 0.0) || !isfinite(d)) bad = k + 1;
      else A[(int64_t)k * ld + k] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    if (bad) break;
    const double inv = 1.0 / A[(int64_t)k * ld + k].x;
    for (int i = k + 1 + tid; i < J; i += kLsSolveThreads) {
      double2 v = A[(int64_t)i * ld + k];
      v = make_double2(v.x * inv, v.y * inv);
      A[(int64_t)i * ld + k] = v;
      lk[i] = v;                            // column k of L, shared for the update
    }
    __syncthreads();
    // trailing lower triangle: A[i][j] -= L[i][k] conj(L[j][k]), k < j <= i; one wave per
    // row (rows interleaved over the waves), lanes over the row's columns (coalesced)
    for (int ii = k + 1 + wave; ii < J; ii += kLsSolveThreads / 64) {
      const double2 lik = lk[ii];
      double2* row = A + (int64_t)ii * ld;
      for (int jj = k + 1 + lane; jj <= ii; jj += 64) {
        const double2 p = cmulc_d(lik, lk[jj]);
        const double2 v = row[jj];
        row[jj] = make_double2(v.x - p.x, v.y - p.y);
      }
    }
    __syncthreads();
  }
  float* cout = coef + (int64_t)set * 2 * J;
  if (bad) {
    for (int i = tid; i < 2 * J; i += kLsSolveThreads) cout[i] = 0.f;
    if (tid == 0) info[set] = bad;
    return;
  }
  // forward: L w = rhs (rhs in column J, overwritten by w)
  for (int k = 0; k < J; ++k) {
    if (tid == 0) {
      const double2 b = A[(int64_t)k * ld + J];
      const double d = A[(int64_t)k * ld + k].x;
      A[(int64_t)k * ld + J] = make_double2(b.x / d, b.y / d);
    }
    __syncthreads();
    const double2 wk = A[(int64_t)k * ld + J];
    for (int i = k + 1 + tid; i < J; i += kLsSolveThreads) {
      const double2 p = cmul_d(A[(int64_t)i * ld + k], wk);
      double2 b = A[(int64_t)i * ld + J];
      A[(int64_t)i * ld + J] = make_double2(b.x - p.x, b.y - p.y);
    }
    __syncthreads();
  }
  // backward: L^H c = w
  for (int k = J - 1; k >= 0; --k) {
    if (tid == 0) {
      const double2 b = A[(int64_t)k * ld + J];
      const double d = A[(int64_t)k * ld + k].x;
      A[(int64_t)k * ld + J] = make_double2(b.x / d, b.y / d);
    }
    __syncthreads();
    const double2 ck = A[(int64_t)k * ld + J];
    for (int i = tid; i < k; i += kLsSolveThreads) {
      // (L^H)[i][k] = conj(L[k][i])
      const double2 p = cmulc_d(ck, A[(int64_t)k * ld + i]);
      double2 b = A[(int64_t)i * ld + J];
      A[(int64_t)i * ld + J] = make_double2(b.x - p.x, b.y - p.y);
    }
    __syncthreads();
  }
  for (int i = tid; i < J; i += kLsSolveThreads) {
    const double2 c = A[(int64_t)i * ld + J];
    cout[2 * i] = (float)c.x;
    cout[2 * i + 1] = (float)c.y;
  }
  if (tid == 0) info[set] = 0;
}

}  // namespace

// ------------------------------------------------------------------ host side
LsDims ls_dims(int K, int M, int L) {
  LsDims d;
  d.J = K * (M + 1) + 2 * (K - 1) * (M + 1) * L;
  // columns padded to a multiple of 64: the last block row / column may be half a block
  d.NCP = round_up(2 * d.J + 2, kLsBlk / 2);
  d.nb = (d.NCP + kLsBlk - 1) / kLsBlk;
  d.nblk = d.nb * (d.nb + 1) / 2;
  d.chunk = kLsChunk;
  return d;
}

int ls_splits(const LsDims& d, int n_tiles, int cus) {
  const int want = (8 * cus + d.nblk - 1) / d.nblk;   // about four rounds of two workgroups per CU
  return std::max(1, std::min(n_tiles, std::min(want, kLsMaxSplits)));
}

static LsGeom geom_of(const dpd_gmp_desc& g) {
  const LsDims d = ls_dims(g.K, g.M, g.L);
  return LsGeom{g.K, g.M, g.L, d.J, d.NCP, d.nb, d.nblk};
}

void launch_ls_gram(const dpd_gmp_desc& g, const StreamTable& st, const float* y, double gi_re,
                    double gi_im, const float* t, int n_splits, double* slots, hipStream_t s) {
  const LsGeom gm = geom_of(g);
  dim3 grid(gm.nblk, n_splits);
  k_ls_gram<<<grid, kLsThreads, 0, s>>>(st, gm, y, gi_re, gi_im, t, n_splits, slots);
}

void launch_ls_reduce(const dpd_gmp_desc& g, const StreamTable& st, int n_splits, const double* slots,
                      double2* normal, hipStream_t s) {
  const LsGeom gm = geom_of(g);
  const int n_sets = st.per_stream ? st.n : 1;
  const int64_t ne = (int64_t)gm.J * (gm.J + 1);
  dim3 rg((unsigned)((ne + 255) / 256), n_sets);
  k_ls_reduce<<<rg, 256, 0, s>>>(st, gm, n_splits, slots, normal);
}

void launch_ls_solve(const dpd_gmp_desc& g, int n_sets, const double2* normal, double ridge,
                     double2* work, float* coef, int* info, hipStream_t s) {
  k_ls_solve<<<n_sets, kLsSolveThreads, 0, s>>>(geom_of(g), normal, ridge, work, coef, info);
}

}  // namespace dpdmi
