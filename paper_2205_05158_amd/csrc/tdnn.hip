// Tuned TDNN DPD kernels for gfx950: the dense layers of the tapped-delay-line
// network (Sec. III-C core, eq. (8) slot) on MFMA, and its reverse mode for direct
// learning (Sec. V-A-2) from the PA-input gradient g_u that the GMP backward kernel
// (eq. (9), gmp.hip) produces.
//
// Formulation.  A layer h_i = tanh(W_i h_{i-1} + b_i) over a wave's block of samples
// is computed transposed, h_i^T = W_i h_{i-1}^T: weights are the MFMA A operand
// (rows = output neurons), activations the B operand (columns = samples).  In the
// accumulator layout a lane owns one sample column and a few neuron rows; those rows
// are exactly a K-slice of the next layer's B operand once the next layer's weights
// are permuted the same way, so activations never leave the registers between
// layers.  The pack kernel writes every weight matrix in that per-lane operand order
// (one 16-byte bf16 or 4-byte fp32 read per lane per MFMA).  The backward chain
// delta_{i-1}^T = W_i^T delta_i^T uses the same trick with a transposed pack.
// dW_i = sum_s delta_i[s] h_{i-1}[s]^T contracts over samples: delta and h are staged
// through LDS (rows = neurons, columns = samples) and the waves accumulate 32x32 dW
// blocks over the tile's samples in MFMA accumulators that stay in registers for the
// workgroup's whole tile range; each (workgroup, stream) slot is written once.
//
// MFMA geometry: BF16 layers use 16x16x32 tiles (16 samples per wave, 64-sample
// workgroup tiles), which halves the per-wave activation state of the deepest model
// relative to 32x32 tiles; FP32 layers use 32x32x2 tiles (32 samples per wave,
// 128-sample workgroup tiles).  The dW contraction always uses 32x32 tiles.
#include "tdnn_kernels.hpp"

namespace dpdmi {

// ------------------------------------------------------------------ host side
// The exact shapes: the paper's three TDNN sizes (Sec. V-A-2) in both precisions.
const TdnnKernels* tdnn_exact(int prec, int T, int H, int NL) {
#define DPD_CASE(P_, T_, H_, NL_) \
  if (prec == P_ && T == T_ && H == H_ && NL == NL_) return &TdnnShape<P_, T_, H_, NL_, false>::table;
  DPD_CASE(DPD_FP32, 4, 20, 2)
  DPD_CASE(DPD_FP32, 10, 64, 3)
  DPD_CASE(DPD_FP32, 16, 128, 4)
  DPD_CASE(DPD_BF16, 4, 20, 2)
  DPD_CASE(DPD_BF16, 10, 64, 3)
  DPD_CASE(DPD_BF16, 16, 128, 4)
#undef DPD_CASE
  return nullptr;
}

// Any other shape with taps <= 32, width <= 128 and 1..4 hidden layers runs on a generic
// instantiation: taps rounded up to 8, 16 or 32 and the width to 32, 64 or 128 (zero
// weights in the padding; the features of the padding taps are masked to zero).
const TdnnKernels* tdnn_generic(int prec, int T, int H, int NL) {
  if (T < 1 || T > 32 || H < 1 || H > 128 || NL < 1 || NL > 4) return nullptr;
  const int tp = T <= 8 ? 8 : (T <= 16 ? 16 : 32);
  const int hp = H <= 32 ? 32 : (H <= 64 ? 64 : 128);
  if (prec == DPD_BF16) {
    if (hp == 32) return tdnn_gen_bf16_32(tp, NL);
    if (hp == 64) return tdnn_gen_bf16_64(tp, NL);
    return tdnn_gen_bf16_128(tp, NL);
  }
  if (prec == DPD_FP32) {
    if (hp == 32) return tdnn_gen_fp32_32(tp, NL);
    if (hp == 64) return tdnn_gen_fp32_64(tp, NL);
    return tdnn_gen_fp32_128(tp, NL);
  }
  return nullptr;
}

bool tdnn_dims(const dpd_tdnn_desc& d, TdnnDims* out) {
  TdnnDims td{};
  td.taps = d.taps;
  td.n_hidden = d.n_hidden;
  td.hidden = d.hidden;
  td.residual = d.residual;
  td.prec = d.precision;
  td.k = tdnn_exact(d.precision, d.taps, d.hidden, d.n_hidden);
  td.generic = td.k == nullptr;
  if (!td.k) td.k = tdnn_generic(d.precision, d.taps, d.hidden, d.n_hidden);
  if (td.k) td.k->dims(&td);
  *out = td;
  return td.k != nullptr;
}

bool tuned_supported(const dpd_tdnn_desc& d, const dpd_gmp_desc* g) {
  TdnnDims td;
  if (!tdnn_dims(d, &td)) return false;
  return !g || gmp_table_coeffs(*g) > 0;
}

void launch_pack(const TdnnDims& td, const float* w, int n_sets, int64_t w_stride, void* pack,
                 hipStream_t s) {
  td.k->pack(td, w, n_sets, w_stride, pack, s);
}

void launch_tdnn_fwd(const TdnnDims& td, const StreamTable& st, const float* x, const void* pack,
                     float* u, int grid, int waves, void* act, hipStream_t s) {
  td.k->fwd(td, st, x, pack, u, grid, waves, td.act_group > 0 ? act : nullptr, s);
}

void set_act_groups(StreamTable& ft, const StreamTable& bt) {
  for (int s = 0; s <= bt.n; ++s) ft.grp0[s] = 4 * bt.tile0[s];
}

void launch_tdnn_bwd(const TdnnDims& td, const StreamTable& st, const float* x, const float* gu,
                     const void* pack, float* slots, int grid, const void* act, hipStream_t s) {
  td.k->bwd(td, st, x, gu, pack, slots, grid, act, s);
}

void launch_dw_finalize(const TdnnDims& td, const StreamTable& st, int grid, const float* slots,
                        const float* inv_r_set, float* dw, hipStream_t s) {
  td.k->finalize(td, st, grid, slots, inv_r_set, dw, s);
}

}  // namespace dpdmi
