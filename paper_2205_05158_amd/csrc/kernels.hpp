// Host-side launchers of the dpdmi kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>

#include "common.hpp"

namespace dpdmi {

// ------------------------------------------------------------------ shared
// (E, R, non-finite count, 0) partial per tile of the stream table (tile = table.tile
// samples).
void launch_nmse_tiles(const StreamTable& st, const float* y, const float* x, float g_re,
                       float g_im, float4* tile_part, hipStream_t s);
// Per-stream and pooled NMSE records (E, R, NMSE dB, non-finite count) from the tile
// partials (rec may be null); optional per-set pooled loss and 1/R per set (inv_r may
// be null).  Two fixed-order stages: chunks of kNmseChunk tiles of one stream, then the
// chunks of each stream; the chunk records go to tile_part[st.n_tiles ..
// st.n_tiles + nmse_chunk_table(st).n_tiles), which the caller provides.
constexpr int kNmseChunk = 256;
StreamTable nmse_chunk_table(const StreamTable& st);
void launch_nmse_final(const StreamTable& st, float4* tile_part, float* rec, float* loss, float* inv_r,
                       hipStream_t s);
// Ideal linear-clipping PA (y = u up to |u| = a, a u / |u| beyond): y of n samples
// (y may equal u), and the cascade pass over the table's tiles: y (may be null), the
// NMSE tile partials and, when gu is not null, g_u = J^T 2 (y - G x).
void launch_clip_fwd(int64_t n, const float* u, float a, float* y, hipStream_t s);
void launch_clip_tiles(const StreamTable& st, const float* x, const float* u, float a, float g_re,
                       float g_im, float4* tile_part, float* gu, float* y, hipStream_t s);
// Symbol MSE of n complex values: out[0] = sum |z - t|^2 / n, out[1] = non-finite count,
// grad (may be null) = scale (z - t); part holds mse_tiles(n) tile partials.
int mse_tiles(int64_t n);
void launch_mse(int64_t n, const float* z, const float* t, float scale, float* grad, float4* part,
                float* out, hipStream_t s);

// ------------------------------------------------------------------ plain path
void launch_plain_features(const float* x, int64_t lo, int64_t c0, int cn, int taps, float* F,
                           hipStream_t s);
void launch_plain_dense(const float* in, int din, const float* W, const float* b, float* out,
                        int dout, int cn, int act, hipStream_t s);
void launch_plain_u(const float* o2, const float* x, int64_t c0, int cn, int residual, float* u,
                    hipStream_t s);
void launch_plain_gmp_fwd(const float* u, int64_t lo, int64_t hi, const float* coef, int K, int M,
                          int L, float* y, hipStream_t s);
void launch_plain_gmp_bwd(const float* u, const float* y, const float* x, int64_t lo, int64_t hi,
                          const float* coef, int K, int M, int L, float g_re, float g_im, float* gu,
                          hipStream_t s);
void launch_plain_delta_out(const float* gu, int64_t c0, int cn, float* d, hipStream_t s);
void launch_plain_dense_bwd(const float* dout, int n_out, const float* W, const float* hin,
                            int n_in, float* din, int cn, hipStream_t s);
void launch_plain_dw(const float* dout, int n_out, const float* hin, int n_in, int cn, int blk,
                     float* part, hipStream_t s);
void launch_plain_dw_accum(const float* part, int nblk, int count, float* acc, hipStream_t s);
void launch_plain_finalize_sets(const float* acc, int taps, int n_hidden, int hidden,
                                int64_t acc_stride, int64_t P, int n_sets, const float* inv_r,
                                float* dw, hipStream_t s);
void launch_fill(float* p, int64_t n, float v, hipStream_t s);

// Adam update of n parameters in place (bias corrections of step `step` >= 1).
void launch_adam(const float* g, float* w, float* m, float* v, int64_t n, int step, double lr,
                 double beta1, double beta2, double eps, int cus, hipStream_t s);

// Least-squares GMP fit (normal equations on the FP64 matrix cores + complex Cholesky).
struct LsDims {
  int J;       // complex coefficients
  int NCP;     // real-embedding columns 2J + 2, padded to a multiple of 64
  int nb;      // 64-column blocks
  int nblk;    // blocks of the upper block triangle
  int chunk;   // samples per basis chunk (stream-table tile)
};
constexpr int kLsMaxSplits = 128;  // sample splits per Gram block (sizes the slots)
constexpr int kLsGramBlk = 128;    // Gram block edge
constexpr int kLsMaxJ = 1024;
LsDims ls_dims(int K, int M, int L);
int ls_splits(const LsDims& d, int n_tiles, int cus);
// st.tile = d.chunk.  slots: (kLsMaxSplits + streams) x nblk x kLsGramBlk^2 doubles; normal
// and work: n_sets x J x (J + 1) complex doubles; coef: n_sets x J complex floats.
void launch_ls_gram(const dpd_gmp_desc& g, const StreamTable& st, const float* y, double gi_re,
                    double gi_im, const float* t, int n_splits, double* slots, hipStream_t s);
void launch_ls_reduce(const dpd_gmp_desc& g, const StreamTable& st, int n_splits, const double* slots,
                      double2* normal, hipStream_t s);
void launch_ls_solve(const dpd_gmp_desc& g, int n_sets, const double2* normal, double ridge,
                     double2* work, float* coef, int* info, hipStream_t s);

// FD-CNN DPD over a batch of items (UE symbol vectors).
struct CnnDims {
  int n_d, side, n_conv, kc;
  int F;           // n_conv side^2 (flattened length)
  int64_t params;  // packed parameter count
};
constexpr int kCnnSplits = 16;    // item splits of the output-weight gradient
constexpr int kCnnConvWg = 1024;  // workgroups of the convolution-gradient pass
CnnDims cnn_dims(int n_d, int side, int n_conv, int kc);
bool cnn_supported(const CnnDims& d);
// h, dpre: workspace [n_items][F]; out, gout: [n_items][n_d][2]; wpart: [kCnnSplits][2 n_d][F + 1];
// cpart: [kCnnConvWg][conv params].  Forward: conv, out.  Reverse: conv, dh, dwout (+ its
// reduction), dwconv.
void launch_cnn_conv(const CnnDims& d, int64_t n_items, const float* s, const float* w, float* h,
                     int cus, hipStream_t st);
void launch_cnn_out(const CnnDims& d, int64_t n_items, const float* h, const float* w, float* out,
                    hipStream_t st);
void launch_cnn_dh(const CnnDims& d, int64_t n_items, const float* gout, const float* w, const float* h,
                   float* dpre, hipStream_t st);
void launch_cnn_dwout(const CnnDims& d, int64_t n_items, const float* gout, const float* h, float* wpart,
                      hipStream_t st);
void launch_cnn_dwout_reduce(const CnnDims& d, const float* wpart, float* dw, hipStream_t st);
void launch_cnn_dwconv(const CnnDims& d, int64_t n_items, const float* s, const float* dpre, float* cpart,
                       float* dw, hipStream_t st);

// ------------------------------------------------------------------ tuned path
struct TdnnDims;
// Launchers of one compiled TDNN shape (tdnn_kernels.hpp): an exact shape, or a generic
// instantiation whose tap count and width come at run time within its compiled bounds.
struct TdnnKernels {
  void (*dims)(TdnnDims* td);
  void (*pack)(const TdnnDims& td, const float* w, int n_sets, int64_t w_stride, void* pack, hipStream_t s);
  void (*fwd)(const TdnnDims& td, const StreamTable& st, const float* x, const void* pack, float* u, int grid,
              int waves, void* act, hipStream_t s);
  void (*bwd)(const TdnnDims& td, const StreamTable& st, const float* x, const float* gu, const void* pack,
              float* slots, int grid, const void* act, hipStream_t s);
  void (*finalize)(const TdnnDims& td, const StreamTable& st, int grid, const float* slots,
                   const float* inv_r_set, float* dw, hipStream_t s);
};
struct TdnnDims {
  int taps, n_hidden, hidden, residual, prec;
  const TdnnKernels* k;   // the compiled shape that runs this model
  bool generic;           // k is a generic instantiation (no exact shape matches)
  int kin;          // 5 * taps
  int hp;           // hidden padded to a multiple of 32 (generic: the compiled width)
  int kin_p;        // layer-1 K padded to the MFMA K step
  int nks1;         // MFMA K steps of layer 1
  int nksh;         // MFMA K steps of a hidden layer
  int tile;         // samples per workgroup tile of the tuned backward kernel
  int fwd_mt;       // samples per wave of the tuned forward kernel
  int fwd_waves;    // default waves per forward workgroup (8, 12 or 16 are compiled)
  int fwd_tile;     // default samples per forward tile (fwd_mt * fwd_waves)
  int64_t pack_bytes;  // bytes of one packed parameter set
  int64_t fwd_lds;     // LDS bytes of the forward kernel at the default tile
  int64_t dw_slot;     // floats per dW slot (natural layout, padded rows and columns)
  int64_t act_group;   // bf16: bytes of the stored activations of one 16-sample group (0: fp32)
};
bool tdnn_dims(const dpd_tdnn_desc& d, TdnnDims* out);
bool tuned_supported(const dpd_tdnn_desc& d, const dpd_gmp_desc* g);

void launch_pack(const TdnnDims& td, const float* w, int n_sets, int64_t w_stride, void* pack,
                 hipStream_t s);
// TDNN forward over the table's tiles (st.tile = td.fwd_mt * waves; waves 8, 12 or 16).
// act (bf16, optional): the hidden activations are also stored per 16-sample group at
// st.grp0 (set_act_groups) for the reverse mode.
void launch_tdnn_fwd(const TdnnDims& td, const StreamTable& st, const float* x, const void* pack,
                     float* u, int grid, int waves, void* act, hipStream_t s);
// Group bases of the stored activations of a forward table ft: 4 groups per 64-sample
// tile of the reverse-mode table bt of the same batch.
void set_act_groups(StreamTable& ft, const StreamTable& bt);
// GMP forward over the table's tiles.
void launch_gmp_fwd(const dpd_gmp_desc& g, const StreamTable& st, const float* u, const float* coef,
                    float* y, hipStream_t s);
// GMP forward + reverse mode over tiles of st.tile samples (256 or 512): y (optional),
// E/R tile partials and g_u = dL/du.  Supported (K, M, L) are those of gmp_dispatch.
// tab: workspace of 2 * J float2 per parameter set (the coefficients and their
// derivative-weighted copy, written first on the same stream).
// Coefficients per parameter set of the reverse-mode kernels' table: J of the order, or of
// the padded order an order without its own instantiation runs on (0: not supported).
int64_t gmp_table_coeffs(const dpd_gmp_desc& g);
void launch_gmp_bwd(const dpd_gmp_desc& g, const StreamTable& st, const float* x, const float* u,
                    const float* coef, float2* tab, float g_re, float g_im, float4* tile_part,
                    float* gu, float* y, hipStream_t s);
// TDNN recompute + reverse mode from g_u: dW partial slots per (workgroup, stream).
// act (bf16: required): the forward's stored activations of the same batch.
void launch_tdnn_bwd(const TdnnDims& td, const StreamTable& st, const float* x, const float* gu,
                     const void* pack, float* slots, int grid, const void* act, hipStream_t s);
void launch_dw_finalize(const TdnnDims& td, const StreamTable& st, int grid, const float* slots,
                        const float* inv_r_set, float* dw, hipStream_t s);

// ------------------------------------------------------------------ spectrum
void launch_welch(const float* y, int64_t n, int nfft, float* seg_part, int n_groups,
                  hipStream_t s);
// sums: workspace float2[kWelchSplits][nfft] (two-stage sum of the group partials)
constexpr int kWelchSplits = 32;
void launch_welch_final(const float* seg_part, int n_groups, int nseg, int nfft, int half_bins,
                        float2* sums, float* psd, float* acpr, hipStream_t s);

// ------------------------------------------------------------------ OFDM downlink
// Batched unitary FFT over rows of n = 2^m points (2 <= n <= 4096): forward
// X_k = n^-1/2 sum x_j e^{-2 pi i jk/n}, inverse with +i.  in may equal out.
bool fft_size_ok(int n);
void launch_fft(const float* in, float* out, int n, int64_t rows, bool inverse, int cus, hipStream_t s);

// FD-NN network dims: F = 2 U (L4+1) <= 64 inputs, hidden <= 32, 1 or 2 hidden layers.
struct NnDims {
  int n_fft, users, memory, hidden, n_hidden;
  int params;        // packed parameter count
  int part_floats;   // floats of one workgroup's padded dW partial (widest layout)
  int mid_floats;    // floats of the reduction's split sums
};
constexpr int kFdnnMaxGroups = 2048;   // backward workgroups (partials) at most
NnDims nn_dims(int n_fft, int users, int memory, int hidden, int n_hidden);
bool nn_supported(const NnDims& d);
int fdnn_bwd_groups(int cus);   // backward grid for `cus` CUs (<= kFdnnMaxGroups partials)
// td, o_td: [n_sym][U][N] complex time samples.
void launch_fdnn_fwd(const NnDims& d, int64_t n_sym, const float* td, const float* w, float* o_td, int cus,
                     hipStream_t s);
// g_td: time-sample gradients [n_sym][U][N]; part: kFdnnMaxGroups * part_floats floats
// (one partial per backward workgroup) followed by mid_floats.  The reduction writes dw.
void launch_fdnn_bwd(const NnDims& d, int64_t n_sym, const float* td, const float* g_td, const float* w,
                     float* part, int cus, hipStream_t s);
void launch_fdnn_reduce(const NnDims& d, int64_t n_sym, float* part, float* dw, int cus, hipStream_t s);
// ZF: pt [n_ch][N][B][U] (data subcarriers only unless all_bins), trace double [n_ch][N],
// alpha [n_ch].  U <= 8, B <= 256, T <= 64.
void launch_zf(const float* h_est, int N, int n_d, int all_bins, int U, int B, int T, int n_ch, float p_total,
               float* pt, double* trace, float* alpha, hipStream_t s);
void launch_precode(const float* pt, const float* alpha, const float* sym, int N, int n_d, int U, int B,
                    int n_sym, int spc, int all_bins, float* x, hipStream_t s);
// true channel on the data subcarriers: hd [n_ch][n_d][U][B]
void launch_chan_data(const float* h, int N, int n_d, int U, int B, int T, int n_ch, float* hd, hipStream_t s);
// rows = n_sym * B rows of x [n_sym][B][N] -> y_fd (same layout); dpd may be null.
void launch_link_pa(const float* x, int N, int B, int64_t rows, const float* dpd, const dpd_gmp_desc* dd,
                    const float* pa, const dpd_gmp_desc& pd, float* y_fd, int cus, hipStream_t s);
// Reverse mode of the link without a DPD: g_r [n_sym][U][n_d] -> g_y (workspace,
// [n_sym][B][N]) -> g_x [n_sym][B][N]; hd as for the receiver.
void launch_link_rx_bwd(const float* hd, const float* alpha, float g_re, float g_im, const float* g_r, int N, int n_d,
                        int U, int B, int n_sym, int spc, float* g_y, hipStream_t s);
void launch_link_pa_bwd(const float* x, const float* g_y, int N, int B, int n_sym, const float* pa,
                        const dpd_gmp_desc& pd, float* g_x, int cus, hipStream_t s);
void launch_precode_bwd(const float* pt, const float* alpha, const float* g_x, int N, int n_d, int U, int B,
                        int n_sym, int spc, int all_bins, float* g_s, hipStream_t s);
int64_t link_rx_parts(int n_d, int n_sym);   // int32 partial counts of U entries each
void launch_link_rx(const float* y_fd, const float* hd, const float* alpha, float g_re, float g_im,
                    const float* noise, const int32_t* tx, int N, int n_d, int U, int B, int n_sym, int spc,
                    int qam_m, float* r_out, int32_t* err_part, int64_t* errors, hipStream_t s);

}  // namespace dpdmi
