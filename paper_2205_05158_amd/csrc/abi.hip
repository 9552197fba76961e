// dpdmi C ABI: host-side validation, workspace layout and dispatch.  Every
// argument is checked before the first HIP call; nothing is allocated; all work
// goes onto the caller's stream.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace dpdmi {
void launch_plain_finalize_sets(const float* acc, int taps, int n_hidden, int hidden,
                                int64_t acc_stride, int64_t P, int n_sets, const float* inv_r,
                                float* dw, hipStream_t s);
}

using namespace dpdmi;

// Scratch of cascade_nmse_noalloc: the per-tile NMSE partials (E, R, non-finite count) and
// the final pass's per-chunk records, DPD_NOALLOC_NMSE_MAX_TILES records in all, in a
// static device array (each
// device that runs the library holds its own copy until the process ends).  In host code
// this name is only a stand-in for the symbol: kernels and runtime calls get the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float4 scratch[DPD_NOALLOC_NMSE_MAX_TILES];

namespace {

constexpr int kNmseTile = 256;        // tile of the stand-alone NMSE pass
constexpr int kPlainChunk = 1 << 17;  // samples per chunk of the plain path
constexpr int kPlainDwBlock = 2048;   // samples per split-K block of the plain dW
constexpr int kMaxGrid = 512;         // persistent workgroups (sizes the dW slots)
constexpr int kGmpTile = 128;         // table tile handed to the stand-alone GMP pass
constexpr int kClipTile = 2048;       // tile of the clipping-PA cascade pass

struct Problem {
  int S = 0, n_sets = 0, per_stream = 0;
  int64_t n_total = 0, max_len = 0;
  int64_t off[DPD_MAX_STREAMS + 1];
};

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

dpd_status check_batch(const dpd_batch* b, Problem* p) {
  if (!b || !b->offsets_host) return DPD_ERR_NULL;
  if (b->n_streams < 1 || b->n_streams > DPD_MAX_STREAMS) return DPD_ERR_SHAPE;
  if (b->per_stream_params != 0 && b->per_stream_params != 1) return DPD_ERR_SHAPE;
  if (b->offsets_host[0] != 0) return DPD_ERR_SHAPE;
  p->S = b->n_streams;
  p->per_stream = b->per_stream_params;
  p->n_sets = p->per_stream ? p->S : 1;
  p->max_len = 0;
  for (int s = 0; s <= p->S; ++s) {
    p->off[s] = b->offsets_host[s];
    if (s > 0) {
      int64_t len = p->off[s] - p->off[s - 1];
      if (len < 1) return DPD_ERR_SHAPE;
      if (len > p->max_len) p->max_len = len;
    }
  }
  p->n_total = p->off[p->S];
  if (p->n_total > (int64_t)1 << 40) return DPD_ERR_SHAPE;
  return DPD_OK;
}

dpd_status check_tdnn(const dpd_tdnn_desc* d) {
  if (!d) return DPD_ERR_NULL;
  if (d->taps < 1 || d->taps > DPD_MAX_TAPS) return DPD_ERR_SHAPE;
  if (d->n_hidden < 1 || d->n_hidden > DPD_MAX_LAYERS) return DPD_ERR_SHAPE;
  if (d->hidden < 1 || d->hidden > DPD_MAX_HIDDEN) return DPD_ERR_SHAPE;
  if (d->residual != 0 && d->residual != 1) return DPD_ERR_SHAPE;
  if (d->precision != DPD_FP32 && d->precision != DPD_BF16) return DPD_ERR_SHAPE;
  if (d->impl != DPD_IMPL_TUNED && d->impl != DPD_IMPL_PLAIN) return DPD_ERR_SHAPE;
  if (d->impl == DPD_IMPL_PLAIN && d->precision != DPD_FP32) return DPD_ERR_UNSUPPORTED;
  if (d->impl == DPD_IMPL_TUNED && !tuned_supported(*d, nullptr)) return DPD_ERR_UNSUPPORTED;
  return DPD_OK;
}

dpd_status check_gmp(const dpd_gmp_desc* g) {
  if (!g) return DPD_ERR_NULL;
  if (g->K < 1 || g->K > DPD_MAX_GMP_K) return DPD_ERR_SHAPE;
  if (g->M < 0 || g->M > DPD_MAX_GMP_M) return DPD_ERR_SHAPE;
  if (g->L < 0 || g->L > DPD_MAX_GMP_L) return DPD_ERR_SHAPE;
  return DPD_OK;
}

int64_t param_count(const dpd_tdnn_desc& d) {
  int64_t din = 5 * (int64_t)d.taps, H = d.hidden;
  return H * din + H + (int64_t)(d.n_hidden - 1) * (H * H + H) + 2 * H + 2;
}
int64_t coeff_count(const dpd_gmp_desc& g) {
  return (int64_t)g.K * (g.M + 1) + 2 * (int64_t)(g.K - 1) * (g.M + 1) * g.L;
}

StreamTable make_table(const Problem& p, int tile) {
  StreamTable st;
  memset(&st, 0, sizeof(st));
  st.n = p.S;
  st.per_stream = p.per_stream;
  st.tile = tile;
  int32_t t = 0;
  for (int s = 0; s < p.S; ++s) {
    st.off[s] = p.off[s];
    st.tile0[s] = t;
    t += (int32_t)ceil_div64(p.off[s + 1] - p.off[s], tile);
  }
  st.off[p.S] = p.off[p.S];
  st.tile0[p.S] = t;
  st.n_tiles = t;
  return st;
}

int device_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

// ------------------------------------------------------------ launch shapes
// The tuned path's run-time shape choices (dpd_tune): forward waves per workgroup (tile
// = fwd_mt x waves samples) and workgroups per CU, backward workgroups per CU, GMP
// reverse-mode tile.  Defaults: the compiled default forward tile with as many
// workgroups per CU as fit in LDS (at most 2), 2 backward workgroups per CU, 256-sample
// GMP tiles.
constexpr int kTuneFwdWaves[] = {8, 12, 16};
constexpr int kTuneGmpTiles[] = {256, 512};
constexpr int kTuneMaxFwdPerCu = 4, kTuneMaxBwdPerCu = 2;

dpd_tune default_tune(const TdnnDims& td) {
  dpd_tune t;
  t.fwd_waves = td.fwd_waves;
  t.fwd_wg_per_cu = (int)std::max<int64_t>(1, std::min<int64_t>(2, (160 * 1024) / (td.fwd_lds + 1024)));
  t.bwd_wg_per_cu = 2;
  t.gmp_tile = 256;
  return t;
}

bool tune_valid(const dpd_tune& t) {
  bool w = false, g = false;
  for (int v : kTuneFwdWaves) w = w || t.fwd_waves == v;
  for (int v : kTuneGmpTiles) g = g || t.gmp_tile == v;
  return w && g && t.fwd_wg_per_cu >= 1 && t.fwd_wg_per_cu <= kTuneMaxFwdPerCu &&
         t.bwd_wg_per_cu >= 1 && t.bwd_wg_per_cu <= kTuneMaxBwdPerCu;
}

// Process-wide table problem -> shape.  A problem is the TDNN descriptor, the GMP
// descriptor (zeros when none) and the batch signature (streams, parameter mode, total
// and longest length).
typedef std::array<int64_t, 13> TuneKey;
TuneKey tune_key(const dpd_tdnn_desc& d, const dpd_gmp_desc* g, const Problem& p) {
  return TuneKey{d.precision, d.taps, d.hidden, d.n_hidden, d.residual, d.impl,
                 g ? g->K : 0, g ? g->M : 0, g ? g->L : 0, p.S, p.per_stream, p.n_total, p.max_len};
}
struct TuneTable {
  std::mutex mu;
  std::map<TuneKey, dpd_tune> map;
};
TuneTable& tune_table() {
  static TuneTable t;
  return t;
}
dpd_tune lookup_tune(const dpd_tdnn_desc& d, const dpd_gmp_desc* g, const Problem& p,
                     const TdnnDims& td) {
  TuneTable& t = tune_table();
  std::lock_guard<std::mutex> lock(t.mu);
  auto it = t.map.find(tune_key(d, g, p));
  return it == t.map.end() ? default_tune(td) : it->second;
}
void store_tune(const dpd_tdnn_desc& d, const dpd_gmp_desc* g, const Problem& p, const dpd_tune* v) {
  TuneTable& t = tune_table();
  std::lock_guard<std::mutex> lock(t.mu);
  if (v) t.map[tune_key(d, g, p)] = *v;
  else t.map.erase(tune_key(d, g, p));
}

int fwd_grid(const dpd_tune& t, const StreamTable& tab) {
  return std::min(tab.n_tiles, t.fwd_wg_per_cu * device_cus());
}
int bwd_grid(const dpd_tune& t, const StreamTable& tab) {
  return std::min(tab.n_tiles, std::min(kMaxGrid, t.bwd_wg_per_cu * device_cus()));
}

// ------------------------------------------------------------ workspace layout
struct Ws {
  size_t tile_part = 0, inv_r = 0, loss_tmp = 0, u_buf = 0, y_buf = 0, gu_buf = 0, gmp_tab = 0;
  size_t act = 0, part = 0, acc = 0, pack = 0, slots = 0, hact = 0, total = 0;
  int64_t act_floats_per_sample = 0;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Ws ws_layout(const dpd_tdnn_desc* d, const dpd_gmp_desc* g, const Problem& p) {

  Ws w;
  size_t pos = 0;
  auto take = [&](size_t bytes) { size_t at = pos; pos = align_up(pos + bytes); return at; };
  int64_t max_tiles = p.n_total / 32 + p.S + 1;   // any tile size >= 32
  int64_t max_chunks = max_tiles / kNmseChunk + p.S + 1;   // the final pass's first stage
  w.tile_part = take(sizeof(float4) * (max_tiles + max_chunks));
  w.inv_r = take(sizeof(float) * p.n_sets);
  w.loss_tmp = take(sizeof(float) * p.n_sets);
  w.u_buf = take(sizeof(float2) * p.n_total);
  w.y_buf = take(sizeof(float2) * p.n_total);
  if (d && d->impl == DPD_IMPL_PLAIN) {
    int64_t H = d->hidden, din = 5 * (int64_t)d->taps;
    int64_t ch = kPlainChunk;
    w.gu_buf = take(sizeof(float2) * p.n_total);
    w.act_floats_per_sample = din + H * d->n_hidden + 2 + 2 * std::max<int64_t>(H, 2);
    w.act = take(sizeof(float) * ch * w.act_floats_per_sample);
    int64_t maxl = std::max(H * (din + 1), std::max(H * (H + 1), 2 * (H + 1)));
    w.part = take(sizeof(float) * (ch / kPlainDwBlock + 1) * maxl);
    w.acc = take(sizeof(float) * p.n_sets * param_count(*d));
  } else if (d) {
    TdnnDims td;
    tdnn_dims(*d, &td);
    w.pack = take((size_t)td.pack_bytes * p.n_sets);
    w.slots = take(sizeof(float) * (size_t)td.dw_slot * (kMaxGrid + p.S));
    w.gu_buf = take(sizeof(float2) * p.n_total);
    if (g) w.gmp_tab = take(sizeof(float2) * 2 * (size_t)std::max<int64_t>(gmp_table_coeffs(*g), 1) * p.n_sets);
    // bf16: the forward's hidden activations for the reverse mode, 4 groups of 16 samples
    // per 64-sample reverse-mode tile
    if (td.act_group > 0) w.hact = take((size_t)td.act_group * 4 * (size_t)make_table(p, td.tile).n_tiles);
  }
  w.total = pos;
  return w;
}

template <class T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off); }

dpd_status launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DPD_OK : DPD_ERR_LAUNCH;
}

// ------------------------------------------------------------ opt-in kernel timing
// When enabled, every kernel launch the library makes is bracketed by two HIP
// events recorded on the caller's stream; dpd_profile_report() waits for them and
// returns per-kernel counts and total milliseconds.  Disabled by default: then no
// event is created and nothing is recorded.
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
struct Prof {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> recs;
};
Prof& prof() {
  static Prof p;
  return p;
}

struct ProfScope {
  hipStream_t s;
  hipEvent_t b = nullptr;
  bool active = false;
  std::string name;
  ProfScope(const char* n, hipStream_t st) : s(st), name(n) {
    Prof& p = prof();
    std::lock_guard<std::mutex> lock(p.mu);
    if (!p.on) return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    (void)hipEventRecord(a, s);
    p.recs.push_back({name, a, b});
    active = true;
  }
  ~ProfScope() {
    if (active) (void)hipEventRecord(b, s);
  }
};
#define DPD_PROF(name) ProfScope _prof_scope_##__LINE__(name, stream)

// ------------------------------------------------------------ plain path pieces
void plain_forward(const dpd_tdnn_desc& d, const Problem& p, const float* x, const float* w,
                   float* u, const Ws& L, void* ws, hipStream_t s) {
  int64_t P = param_count(d);
  int H = d.hidden, din = 5 * d.taps;
  float* act = at<float>(ws, L.act);
  for (int st = 0; st < p.S; ++st) {
    const float* wp = w + (p.per_stream ? st * P : 0);
    for (int64_t c0 = p.off[st]; c0 < p.off[st + 1]; c0 += kPlainChunk) {
      int cn = (int)std::min<int64_t>(kPlainChunk, p.off[st + 1] - c0);
      float* F = act;
      launch_plain_features(x, p.off[st], c0, cn, d.taps, F, s);
      const float* in = F;
      int k_in = din;
      float* h = F + (int64_t)kPlainChunk * din;
      const float* wl = wp;
      for (int i = 0; i < d.n_hidden; ++i) {
        launch_plain_dense(in, k_in, wl, wl + (int64_t)H * k_in, h, H, cn, 1, s);
        wl += (int64_t)H * k_in + H;
        in = h;
        k_in = H;
        h += (int64_t)kPlainChunk * H;
      }
      launch_plain_dense(in, k_in, wl, wl + 2 * (int64_t)k_in, h, 2, cn, 0, s);
      launch_plain_u(h, x, c0, cn, d.residual, u, s);
    }
  }
}

void plain_gmp_forward(const dpd_gmp_desc& g, const Problem& p, const float* u, const float* coef,
                       float* y, hipStream_t s) {
  int64_t J = coeff_count(g);
  for (int st = 0; st < p.S; ++st)
    launch_plain_gmp_fwd(u, p.off[st], p.off[st + 1], coef + (p.per_stream ? st * 2 * J : 0), g.K,
                         g.M, g.L, y, s);
}

// g: the GMP PA whose reverse mode gives g_u; null when g_u is already in the workspace
// (the clipping PA's cascade pass writes it there).
void plain_backward(const dpd_tdnn_desc& d, const dpd_gmp_desc* g, const Problem& p,
                    const float* x, const float* w, const float* coef, float g_re, float g_im,
                    const float* u, const float* y, float* dw, const float* inv_r, const Ws& L,
                    void* ws, hipStream_t s) {
  int64_t P = param_count(d);
  int H = d.hidden, din = 5 * d.taps, nl = d.n_hidden;
  float* gu = at<float>(ws, L.gu_buf);
  if (g) {
    const int64_t J = coeff_count(*g);
    for (int st = 0; st < p.S; ++st)
      launch_plain_gmp_bwd(u, y, x, p.off[st], p.off[st + 1], coef + (p.per_stream ? st * 2 * J : 0),
                           g->K, g->M, g->L, g_re, g_im, gu, s);
  }
  float* acc = at<float>(ws, L.acc);
  launch_fill(acc, (int64_t)p.n_sets * P, 0.f, s);
  float* act = at<float>(ws, L.act);
  float* part = at<float>(ws, L.part);
  const int64_t ch = kPlainChunk;
  for (int st = 0; st < p.S; ++st) {
    int set = p.per_stream ? st : 0;
    const float* wp = w + set * P;
    float* accp = acc + set * P;
    for (int64_t c0 = p.off[st]; c0 < p.off[st + 1]; c0 += ch) {
      int cn = (int)std::min<int64_t>(ch, p.off[st + 1] - c0);
      // forward, keeping every activation of the chunk
      float* F = act;
      launch_plain_features(x, p.off[st], c0, cn, d.taps, F, s);
      const float* hs[DPD_MAX_LAYERS + 1];
      const float* wls[DPD_MAX_LAYERS + 1];
      int ins[DPD_MAX_LAYERS + 1];
      hs[0] = F;
      float* h = F + ch * din;
      const float* wl = wp;
      int k_in = din;
      for (int i = 0; i < nl; ++i) {
        wls[i] = wl;
        ins[i] = k_in;
        launch_plain_dense(hs[i], k_in, wl, wl + (int64_t)H * k_in, h, H, cn, 1, s);
        hs[i + 1] = h;
        wl += (int64_t)H * k_in + H;
        k_in = H;
        h += ch * H;
      }
      wls[nl] = wl;
      ins[nl] = H;
      float* dA = h;                       // ping-pong delta buffers
      float* dB = h + ch * std::max(H, 2);
      launch_plain_delta_out(gu, c0, cn, dA, s);
      // layer offsets inside the packed/acc layout
      int64_t loff[DPD_MAX_LAYERS + 1];
      int64_t pos = 0;
      for (int i = 0; i <= nl; ++i) {
        loff[i] = pos;
        int dout = i == nl ? 2 : H;
        pos += (int64_t)dout * (ins[i] + 1);
      }
      int nblk = (cn + kPlainDwBlock - 1) / kPlainDwBlock;
      for (int i = nl; i >= 0; --i) {
        int dout = i == nl ? 2 : H;
        launch_plain_dw(dA, dout, hs[i], ins[i], cn, kPlainDwBlock, part, s);
        launch_plain_dw_accum(part, nblk, dout * (ins[i] + 1), accp + loff[i], s);
        if (i > 0) {
          launch_plain_dense_bwd(dA, dout, wls[i], hs[i], ins[i], dB, cn, s);
          std::swap(dA, dB);
        }
      }
    }
  }
  launch_plain_finalize_sets(acc, d.taps, nl, H, P, P, p.n_sets, inv_r, dw, s);
}

}  // namespace

// =====================================================================================
extern "C" {

int64_t dpd_tdnn_param_count(const dpd_tdnn_desc* tdnn) {
  if (!tdnn || tdnn->taps < 1 || tdnn->hidden < 1 || tdnn->n_hidden < 1) return -1;
  return param_count(*tdnn);
}

int64_t dpd_gmp_coeff_count(const dpd_gmp_desc* gmp) {
  if (check_gmp(gmp) != DPD_OK) return -1;
  return coeff_count(*gmp);
}

dpd_status dpd_workspace_size(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp,
                              const dpd_batch* batch, size_t* bytes_host) {
  if (!bytes_host) return DPD_ERR_NULL;
  Problem p;
  dpd_status st = check_batch(batch, &p);
  if (st != DPD_OK) return st;
  if (tdnn && (st = check_tdnn(tdnn)) != DPD_OK) return st;
  if (gmp && (st = check_gmp(gmp)) != DPD_OK) return st;
  *bytes_host = ws_layout(tdnn, gmp, p).total;
  return DPD_OK;
}

dpd_status dpd_forward(const dpd_tdnn_desc* tdnn, const dpd_batch* batch, const float* x,
                       const float* w, float* u, void* workspace, size_t workspace_bytes,
                       hipStream_t stream) {
  Problem p;
  dpd_status st;
  if ((st = check_tdnn(tdnn)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!x || !w || !u || !workspace) return DPD_ERR_NULL;
  if (!aligned(x, 8) || !aligned(u, 8) || !aligned(w, 4) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  Ws L = ws_layout(tdnn, nullptr, p);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  if (tdnn->impl == DPD_IMPL_PLAIN) {
    DPD_PROF("plain_forward");
    plain_forward(*tdnn, p, x, w, u, L, workspace, stream);
  } else {
    TdnnDims td;
    tdnn_dims(*tdnn, &td);
    void* pack = at<void>(workspace, L.pack);
    { DPD_PROF("pack"); launch_pack(td, w, p.n_sets, param_count(*tdnn), pack, stream); }
    const dpd_tune tn = lookup_tune(*tdnn, nullptr, p, td);
    StreamTable tab = make_table(p, td.fwd_mt * tn.fwd_waves);
    { DPD_PROF("tdnn_fwd"); launch_tdnn_fwd(td, tab, x, pack, u, fwd_grid(tn, tab), tn.fwd_waves, nullptr, stream); }
  }
  return launch_status();
}

dpd_status pa_gmp_forward(const dpd_gmp_desc* gmp, const dpd_batch* batch, const float* u,
                          const float* coef, float* y, hipStream_t stream) {
  Problem p;
  dpd_status st;
  if ((st = check_gmp(gmp)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!u || !coef || !y) return DPD_ERR_NULL;
  if (!aligned(u, 8) || !aligned(y, 8) || !aligned(coef, 4)) return DPD_ERR_ALIGN;
  if (u == y) return DPD_ERR_SHAPE;
  StreamTable tab = make_table(p, kGmpTile);
  { DPD_PROF("gmp_fwd"); launch_gmp_fwd(*gmp, tab, u, coef, y, stream); }
  return launch_status();
}

dpd_status dpd_symbol_mse_workspace_size(int64_t n, size_t* bytes_host) {
  if (!bytes_host) return DPD_ERR_NULL;
  if (n < 1) return DPD_ERR_SHAPE;
  *bytes_host = align_up(sizeof(float4) * (size_t)mse_tiles(n));
  return DPD_OK;
}

dpd_status dpd_symbol_mse(int64_t n, const float* z, const float* t, float* out, float* grad,
                          void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (n < 1) return DPD_ERR_SHAPE;
  if (!z || !t || !out || !workspace) return DPD_ERR_NULL;
  if (!aligned(z, 8) || !aligned(t, 8) || !aligned(out, 4) || (grad && !aligned(grad, 8)) ||
      !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (grad && (grad == z || grad == t)) return DPD_ERR_SHAPE;
  if (workspace_bytes < align_up(sizeof(float4) * (size_t)mse_tiles(n))) return DPD_ERR_WORKSPACE;
  {
    DPD_PROF("symbol_mse");
    launch_mse(n, z, t, (float)(2.0 / (double)n), grad, static_cast<float4*>(workspace), out, stream);
  }
  return launch_status();
}

// Device address of `scratch` on the current device, looked up once per device (with
// that device current) and kept; null if the runtime reports an error.
float4* noalloc_scratch_ptr() {
  static std::mutex mu;
  static float4* addr[64] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    addr[dev] = static_cast<float4*>(p);
  }
  return addr[dev];
}

dpd_status cascade_nmse_noalloc(const dpd_batch* batch, const float* y, const float* x, float g_re,
                                float g_im, float* out, hipStream_t stream) {
  Problem p;
  dpd_status st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!y || !x || !out) return DPD_ERR_NULL;
  if (!aligned(y, 8) || !aligned(x, 8) || !aligned(out, 4)) return DPD_ERR_ALIGN;
  if (!isfinite(g_re) || !isfinite(g_im) || (g_re == 0.f && g_im == 0.f)) return DPD_ERR_SHAPE;
  StreamTable tab = make_table(p, kNmseTile);
  if ((int64_t)tab.n_tiles + nmse_chunk_table(tab).n_tiles > DPD_NOALLOC_NMSE_MAX_TILES)
    return DPD_ERR_WORKSPACE;
  float4* part = noalloc_scratch_ptr();
  if (!part) return DPD_ERR_LAUNCH;
  // every partial the final pass reads is written by the tile pass first: nothing to clear
  { DPD_PROF("nmse_tiles"); launch_nmse_tiles(tab, y, x, g_re, g_im, part, stream); }
  { DPD_PROF("nmse_final"); launch_nmse_final(tab, part, out, nullptr, nullptr, stream); }
  return launch_status();
}

dpd_status dpd_nmse_status(const float* nmse_host, int64_t n_records) {
  if (!nmse_host) return DPD_ERR_NULL;
  if (n_records < 1) return DPD_ERR_SHAPE;
  for (int64_t r = 0; r < n_records; ++r) {
    const float* rec = nmse_host + r * DPD_NMSE_FIELDS;
    // NMSE_dB = -inf is the exact match E = 0 (a finite result); NaN or +inf is not
    if (!(rec[3] == 0.f) || !isfinite(rec[0]) || !isfinite(rec[1]) || isnan(rec[2]) ||
        (isinf(rec[2]) && rec[2] > 0.f))
      return DPD_ERR_NONFINITE;
  }
  return DPD_OK;
}

dpd_status cascade_nmse(const dpd_batch* batch, const float* y, const float* x, float g_re,
                        float g_im, float* out, void* workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  Problem p;
  dpd_status st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!y || !x || !out || !workspace) return DPD_ERR_NULL;
  if (!aligned(y, 8) || !aligned(x, 8) || !aligned(out, 4) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (!isfinite(g_re) || !isfinite(g_im) || (g_re == 0.f && g_im == 0.f)) return DPD_ERR_SHAPE;
  Ws L = ws_layout(nullptr, nullptr, p);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  StreamTable tab = make_table(p, kNmseTile);
  float4* part = at<float4>(workspace, L.tile_part);
  { DPD_PROF("nmse_tiles"); launch_nmse_tiles(tab, y, x, g_re, g_im, part, stream); }
  { DPD_PROF("nmse_final"); launch_nmse_final(tab, part, out, nullptr, nullptr, stream); }
  return launch_status();
}

dpd_status dpd_cascade(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp, const dpd_batch* batch,
                       const float* x, const float* w, const float* coef, float g_re, float g_im,
                       float* u, float* y, float* nmse, float* dw, float* loss, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  Problem p;
  dpd_status st;
  if ((st = check_tdnn(tdnn)) != DPD_OK) return st;
  if ((st = check_gmp(gmp)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!x || !w || !coef || !workspace) return DPD_ERR_NULL;
  if (dw && !loss) return DPD_ERR_NULL;
  if (!aligned(x, 8) || (u && !aligned(u, 8)) || (y && !aligned(y, 8)) || !aligned(w, 4) ||
      !aligned(coef, 4) || (dw && !aligned(dw, 4)) || (loss && !aligned(loss, 4)) ||
      (nmse && !aligned(nmse, 4)) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (!isfinite(g_re) || !isfinite(g_im) || (g_re == 0.f && g_im == 0.f)) return DPD_ERR_SHAPE;
  if (dw && tdnn->impl == DPD_IMPL_TUNED && !tuned_supported(*tdnn, gmp)) return DPD_ERR_UNSUPPORTED;
  Ws L = ws_layout(tdnn, gmp, p);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  float* ubuf = u ? u : at<float>(workspace, L.u_buf);
  float* inv_r = at<float>(workspace, L.inv_r);
  float* lossp = loss ? loss : at<float>(workspace, L.loss_tmp);
  float4* part = at<float4>(workspace, L.tile_part);
  int64_t P = param_count(*tdnn);
  if (tdnn->impl == DPD_IMPL_PLAIN) {
    float* ybuf = y ? y : at<float>(workspace, L.y_buf);
    { DPD_PROF("plain_forward"); plain_forward(*tdnn, p, x, w, ubuf, L, workspace, stream); }
    { DPD_PROF("plain_gmp_fwd"); plain_gmp_forward(*gmp, p, ubuf, coef, ybuf, stream); }
    StreamTable tab = make_table(p, kNmseTile);
    { DPD_PROF("nmse_tiles"); launch_nmse_tiles(tab, ybuf, x, g_re, g_im, part, stream); }
    { DPD_PROF("nmse_final"); launch_nmse_final(tab, part, nmse, lossp, inv_r, stream); }
    if (dw) {
      DPD_PROF("plain_backward");
      plain_backward(*tdnn, gmp, p, x, w, coef, g_re, g_im, ubuf, ybuf, dw, inv_r, L, workspace,
                     stream);
    }
    return launch_status();
  }
  TdnnDims td;
  tdnn_dims(*tdnn, &td);
  void* pack = at<void>(workspace, L.pack);
  { DPD_PROF("pack"); launch_pack(td, w, p.n_sets, P, pack, stream); }
  const dpd_tune tn = lookup_tune(*tdnn, gmp, p, td);
  StreamTable ftab = make_table(p, td.fwd_mt * tn.fwd_waves);
  StreamTable tab = make_table(p, td.tile);
  set_act_groups(ftab, tab);
  void* hact = at<void>(workspace, L.hact);
  { DPD_PROF("tdnn_fwd"); launch_tdnn_fwd(td, ftab, x, pack, ubuf, fwd_grid(tn, ftab), tn.fwd_waves, dw ? hact : nullptr, stream); }
  if (dw) {
    // GMP forward + reverse mode (y, E/R tile partials, g_u), then the TDNN reverse mode
    StreamTable gt = make_table(p, tn.gmp_tile);
    float* gub = at<float>(workspace, L.gu_buf);
    float2* gtab = at<float2>(workspace, L.gmp_tab);
    { DPD_PROF("gmp_bwd"); launch_gmp_bwd(*gmp, gt, x, ubuf, coef, gtab, g_re, g_im, part, gub, y, stream); }
    const int grid = bwd_grid(tn, tab);
    float* slots = at<float>(workspace, L.slots);
    { DPD_PROF("tdnn_bwd"); launch_tdnn_bwd(td, tab, x, gub, pack, slots, grid, hact, stream); }
    { DPD_PROF("nmse_final"); launch_nmse_final(gt, part, nmse, lossp, inv_r, stream); }
    { DPD_PROF("dw_finalize"); launch_dw_finalize(td, tab, grid, slots, inv_r, dw, stream); }
  } else {
    float* ybuf = y ? y : at<float>(workspace, L.y_buf);
    { DPD_PROF("gmp_fwd"); launch_gmp_fwd(*gmp, tab, ubuf, coef, ybuf, stream); }
    StreamTable nt = make_table(p, kNmseTile);
    { DPD_PROF("nmse_tiles"); launch_nmse_tiles(nt, ybuf, x, g_re, g_im, part, stream); }
    { DPD_PROF("nmse_final"); launch_nmse_final(nt, part, nmse, lossp, inv_r, stream); }
  }
  return launch_status();
}

dpd_status dpd_backward(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp, const dpd_batch* batch,
                        const float* x, const float* w, const float* coef, float g_re, float g_im,
                        float* dw, float* loss, void* workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  if (!dw || !loss) return DPD_ERR_NULL;
  return dpd_cascade(tdnn, gmp, batch, x, w, coef, g_re, g_im, nullptr, nullptr, nullptr, dw, loss,
                     workspace, workspace_bytes, stream);
}

dpd_status pa_clip_forward(int64_t n, const float* u, float a_clip, float* y, hipStream_t stream) {
  if (n < 1) return DPD_ERR_SHAPE;
  if (!u || !y) return DPD_ERR_NULL;
  if (!aligned(u, 8) || !aligned(y, 8)) return DPD_ERR_ALIGN;
  if (!(a_clip > 0.f) || !isfinite(a_clip)) return DPD_ERR_SHAPE;
  { DPD_PROF("clip_fwd"); launch_clip_fwd(n, u, a_clip, y, stream); }
  return launch_status();
}

dpd_status dpd_cascade_clip(const dpd_tdnn_desc* tdnn, const dpd_batch* batch, const float* x,
                            const float* w, float a_clip, float g_re, float g_im, float* u, float* y,
                            float* nmse, float* dw, float* loss, void* workspace,
                            size_t workspace_bytes, hipStream_t stream) {
  Problem p;
  dpd_status st;
  if ((st = check_tdnn(tdnn)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!x || !w || !workspace) return DPD_ERR_NULL;
  if (dw && !loss) return DPD_ERR_NULL;
  if (!aligned(x, 8) || (u && !aligned(u, 8)) || (y && !aligned(y, 8)) || !aligned(w, 4) ||
      (dw && !aligned(dw, 4)) || (loss && !aligned(loss, 4)) || (nmse && !aligned(nmse, 4)) ||
      !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (!isfinite(g_re) || !isfinite(g_im) || (g_re == 0.f && g_im == 0.f)) return DPD_ERR_SHAPE;
  if (!(a_clip > 0.f) || !isfinite(a_clip)) return DPD_ERR_SHAPE;
  Ws L = ws_layout(tdnn, nullptr, p);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  float* ubuf = u ? u : at<float>(workspace, L.u_buf);
  float* inv_r = at<float>(workspace, L.inv_r);
  float* lossp = loss ? loss : at<float>(workspace, L.loss_tmp);
  float4* part = at<float4>(workspace, L.tile_part);
  float* gub = dw ? at<float>(workspace, L.gu_buf) : nullptr;
  StreamTable ct = make_table(p, kClipTile);
  if (tdnn->impl == DPD_IMPL_PLAIN) {
    { DPD_PROF("plain_forward"); plain_forward(*tdnn, p, x, w, ubuf, L, workspace, stream); }
    { DPD_PROF("clip_tiles"); launch_clip_tiles(ct, x, ubuf, a_clip, g_re, g_im, part, gub, y, stream); }
    { DPD_PROF("nmse_final"); launch_nmse_final(ct, part, nmse, lossp, inv_r, stream); }
    if (dw) {
      DPD_PROF("plain_backward");
      plain_backward(*tdnn, nullptr, p, x, w, nullptr, g_re, g_im, ubuf, y, dw, inv_r, L, workspace, stream);
    }
    return launch_status();
  }
  TdnnDims td;
  tdnn_dims(*tdnn, &td);
  void* pack = at<void>(workspace, L.pack);
  { DPD_PROF("pack"); launch_pack(td, w, p.n_sets, param_count(*tdnn), pack, stream); }
  const dpd_tune tn = lookup_tune(*tdnn, nullptr, p, td);
  StreamTable ftab = make_table(p, td.fwd_mt * tn.fwd_waves);
  set_act_groups(ftab, make_table(p, td.tile));
  void* hact = at<void>(workspace, L.hact);
  { DPD_PROF("tdnn_fwd"); launch_tdnn_fwd(td, ftab, x, pack, ubuf, fwd_grid(tn, ftab), tn.fwd_waves, dw ? hact : nullptr, stream); }
  { DPD_PROF("clip_tiles"); launch_clip_tiles(ct, x, ubuf, a_clip, g_re, g_im, part, gub, y, stream); }
  { DPD_PROF("nmse_final"); launch_nmse_final(ct, part, nmse, lossp, inv_r, stream); }
  if (dw) {
    StreamTable tab = make_table(p, td.tile);
    const int grid = bwd_grid(tn, tab);
    float* slots = at<float>(workspace, L.slots);
    { DPD_PROF("tdnn_bwd"); launch_tdnn_bwd(td, tab, x, gub, pack, slots, grid, hact, stream); }
    { DPD_PROF("dw_finalize"); launch_dw_finalize(td, tab, grid, slots, inv_r, dw, stream); }
  }
  return launch_status();
}

dpd_status dpd_tune_get(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp, const dpd_batch* batch,
                        dpd_tune* out_host) {
  Problem p;
  dpd_status st;
  if (!out_host) return DPD_ERR_NULL;
  if ((st = check_tdnn(tdnn)) != DPD_OK) return st;
  if (gmp && (st = check_gmp(gmp)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (tdnn->impl != DPD_IMPL_TUNED) return DPD_ERR_UNSUPPORTED;
  TdnnDims td;
  tdnn_dims(*tdnn, &td);
  *out_host = lookup_tune(*tdnn, gmp, p, td);
  return DPD_OK;
}

dpd_status dpd_tune_set(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp, const dpd_batch* batch,
                        const dpd_tune* tune_host) {
  Problem p;
  dpd_status st;
  if ((st = check_tdnn(tdnn)) != DPD_OK) return st;
  if (gmp && (st = check_gmp(gmp)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (tdnn->impl != DPD_IMPL_TUNED) return DPD_ERR_UNSUPPORTED;
  if (tune_host && !tune_valid(*tune_host)) return DPD_ERR_SHAPE;
  store_tune(*tdnn, gmp, p, tune_host);
  return DPD_OK;
}

dpd_status dpd_autotune(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp, const dpd_batch* batch,
                        const float* x, const float* w, const float* coef, float g_re, float g_im,
                        int32_t reps, void* workspace, size_t workspace_bytes, hipStream_t stream,
                        dpd_tune* out_host) {
  Problem p;
  dpd_status st;
  if ((st = check_tdnn(tdnn)) != DPD_OK) return st;
  if ((st = check_gmp(gmp)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!x || !w || !coef || !workspace || !out_host) return DPD_ERR_NULL;
  if (!aligned(x, 8) || !aligned(w, 4) || !aligned(coef, 4) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (!isfinite(g_re) || !isfinite(g_im) || (g_re == 0.f && g_im == 0.f)) return DPD_ERR_SHAPE;
  if (reps < 1 || reps > 1000) return DPD_ERR_SHAPE;
  if (tdnn->impl != DPD_IMPL_TUNED || !tuned_supported(*tdnn, gmp)) return DPD_ERR_UNSUPPORTED;
  Ws L = ws_layout(tdnn, gmp, p);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  TdnnDims td;
  tdnn_dims(*tdnn, &td);
  void* pack = at<void>(workspace, L.pack);
  float* ubuf = at<float>(workspace, L.u_buf);
  float* gub = at<float>(workspace, L.gu_buf);
  float2* gtab = at<float2>(workspace, L.gmp_tab);
  float4* part = at<float4>(workspace, L.tile_part);
  float* slots = at<float>(workspace, L.slots);
  const dpd_tune def = default_tune(td);
  const StreamTable btab = make_table(p, td.tile);
  void* hact = at<void>(workspace, L.hact);

  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return DPD_ERR_LAUNCH;
  }
  bool failed = false;
  // milliseconds of reps back-to-back runs of fn on the caller's stream
  auto time_ms = [&](auto&& fn) {
    float ms = 1e30f;
    if (failed) return ms;
    fn();   // untimed first run
    if (hipEventRecord(ev[0], stream) != hipSuccess) { failed = true; return ms; }
    for (int r = 0; r < reps; ++r) fn();
    if (hipEventRecord(ev[1], stream) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
        hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess || hipGetLastError() != hipSuccess) {
      failed = true;
      ms = 1e30f;
    }
    return ms;
  };

  // inputs of each timed kernel: packed weights, u, g_u (default shapes)
  launch_pack(td, w, p.n_sets, param_count(*tdnn), pack, stream);
  {
    StreamTable ft = make_table(p, td.fwd_mt * def.fwd_waves);
    set_act_groups(ft, btab);
    launch_tdnn_fwd(td, ft, x, pack, ubuf, fwd_grid(def, ft), def.fwd_waves, hact, stream);
    StreamTable gt = make_table(p, def.gmp_tile);
    launch_gmp_bwd(*gmp, gt, x, ubuf, coef, gtab, g_re, g_im, part, gub, nullptr, stream);
  }
  dpd_tune best = def;
  float best_ms = 1e30f;
  for (int wv : kTuneFwdWaves)
    for (int pc = 1; pc <= kTuneMaxFwdPerCu; ++pc) {
      dpd_tune c = def;
      c.fwd_waves = wv;
      c.fwd_wg_per_cu = pc;
      StreamTable ft = make_table(p, td.fwd_mt * wv);
      set_act_groups(ft, btab);
      if (pc > 1 && (pc - 1) * device_cus() >= ft.n_tiles) continue;   // same grid as pc - 1
      const float ms = time_ms([&] { launch_tdnn_fwd(td, ft, x, pack, ubuf, fwd_grid(c, ft), wv, hact, stream); });
      if (ms < best_ms) { best_ms = ms; best.fwd_waves = wv; best.fwd_wg_per_cu = pc; }
    }
  best_ms = 1e30f;
  for (int gtile : kTuneGmpTiles) {
    StreamTable gt = make_table(p, gtile);
    const float ms = time_ms([&] {
      launch_gmp_bwd(*gmp, gt, x, ubuf, coef, gtab, g_re, g_im, part, gub, nullptr, stream);
    });
    if (ms < best_ms) { best_ms = ms; best.gmp_tile = gtile; }
  }
  best_ms = 1e30f;
  for (int pc = 1; pc <= kTuneMaxBwdPerCu; ++pc) {
    dpd_tune c = def;
    c.bwd_wg_per_cu = pc;
    if (pc > 1 && (pc - 1) * device_cus() >= btab.n_tiles) continue;
    const float ms = time_ms([&] { launch_tdnn_bwd(td, btab, x, gub, pack, slots, bwd_grid(c, btab), hact, stream); });
    if (ms < best_ms) { best_ms = ms; best.bwd_wg_per_cu = pc; }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (failed) return DPD_ERR_LAUNCH;
  store_tune(*tdnn, gmp, p, &best);
  *out_host = best;
  return DPD_OK;
}

dpd_status dpd_adam_step(const float* grad, float* w, float* m, float* v, int64_t n, int32_t step,
                         double lr, double beta1, double beta2, double eps, hipStream_t stream) {
  if (!grad || !w || !m || !v) return DPD_ERR_NULL;
  if (n < 1 || n > ((int64_t)1 << 40) || step < 1) return DPD_ERR_SHAPE;
  if (!isfinite(lr) || !isfinite(eps) || eps < 0.0 || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0))
    return DPD_ERR_SHAPE;
  if (!aligned(grad, 4) || !aligned(w, 4) || !aligned(m, 4) || !aligned(v, 4)) return DPD_ERR_ALIGN;
  // the four vectors must not overlap (each is n floats)
  const uintptr_t lo[4] = {(uintptr_t)grad, (uintptr_t)w, (uintptr_t)m, (uintptr_t)v};
  const uintptr_t len = (uintptr_t)n * sizeof(float);
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (lo[i] < lo[j] + len && lo[j] < lo[i] + len) return DPD_ERR_SHAPE;
  { DPD_PROF("adam"); launch_adam(grad, w, m, v, n, step, lr, beta1, beta2, eps, device_cus(), stream); }
  return launch_status();
}

}  // extern "C"

namespace {
struct LsWs {
  size_t slots = 0, normal = 0, work = 0, total = 0;
};
LsWs ls_ws_layout(const dpd_gmp_desc& g, const Problem& p) {
  const LsDims d = ls_dims(g.K, g.M, g.L);
  LsWs w;
  size_t pos = 0;
  auto take = [&](size_t bytes) { size_t at = pos; pos = align_up(pos + bytes); return at; };
  w.slots = take(sizeof(double) * (size_t)(kLsMaxSplits + p.S) * d.nblk * kLsGramBlk * kLsGramBlk);
  w.normal = take(sizeof(double2) * (size_t)p.n_sets * d.J * (d.J + 1));
  w.work = take(sizeof(double2) * (size_t)p.n_sets * d.J * (d.J + 1));
  w.total = pos;
  return w;
}
dpd_status check_ls_gmp(const dpd_gmp_desc* gmp) {
  dpd_status st = check_gmp(gmp);
  if (st != DPD_OK) return st;
  return coeff_count(*gmp) <= kLsMaxJ ? DPD_OK : DPD_ERR_UNSUPPORTED;
}
}  // namespace

extern "C" {

dpd_status gmp_ls_workspace_size(const dpd_gmp_desc* gmp, const dpd_batch* batch, size_t* bytes_host) {
  Problem p;
  dpd_status st;
  if (!bytes_host) return DPD_ERR_NULL;
  if ((st = check_ls_gmp(gmp)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  *bytes_host = ls_ws_layout(*gmp, p).total;
  return DPD_OK;
}

dpd_status gmp_ls_fit(const dpd_gmp_desc* gmp, const dpd_batch* batch, const float* y, float g_re,
                      float g_im, const float* t, double ridge, float* coef, int32_t* info,
                      double* normal_out, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  Problem p;
  dpd_status st;
  if ((st = check_ls_gmp(gmp)) != DPD_OK) return st;
  if ((st = check_batch(batch, &p)) != DPD_OK) return st;
  if (!y || !t || !coef || !info || !workspace) return DPD_ERR_NULL;
  if (!aligned(y, 8) || !aligned(t, 8) || !aligned(coef, 4) || !aligned(info, 4) ||
      (normal_out && !aligned(normal_out, 16)) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (!isfinite(g_re) || !isfinite(g_im) || (g_re == 0.f && g_im == 0.f)) return DPD_ERR_SHAPE;
  if (!isfinite(ridge) || ridge < 0.0) return DPD_ERR_SHAPE;
  const LsWs L = ls_ws_layout(*gmp, p);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  const LsDims d = ls_dims(gmp->K, gmp->M, gmp->L);
  const StreamTable tab = make_table(p, d.chunk);
  const int splits = ls_splits(d, tab.n_tiles, device_cus());
  const double gr = g_re, gi = g_im, m2 = gr * gr + gi * gi;   // 1 / G
  double2* normal = normal_out ? reinterpret_cast<double2*>(normal_out) : at<double2>(workspace, L.normal);
  double* slots = at<double>(workspace, L.slots);
  { DPD_PROF("ls_gram"); launch_ls_gram(*gmp, tab, y, gr / m2, -gi / m2, t, splits, slots, stream); }
  { DPD_PROF("ls_reduce"); launch_ls_reduce(*gmp, tab, splits, slots, normal, stream); }
  {
    DPD_PROF("ls_solve");
    launch_ls_solve(*gmp, p.n_sets, normal, ridge, at<double2>(workspace, L.work), coef, info, stream);
  }
  return launch_status();
}

}  // extern "C"

namespace {
struct CnnWs {
  size_t h = 0, dpre = 0, wpart = 0, cpart = 0, total = 0;
};
bool cnn_check(const dpd_fdcnn_desc* d, CnnDims* out) {
  if (!d) return false;
  const CnnDims c = cnn_dims(d->n_d, d->side, d->n_conv, d->kc);
  if (!cnn_supported(c)) return false;
  *out = c;
  return true;
}
CnnWs cnn_ws_layout(const CnnDims& d, int64_t n_items) {
  CnnWs w;
  size_t pos = 0;
  auto take = [&](size_t bytes) { size_t at = pos; pos = align_up(pos + bytes); return at; };
  w.h = take(sizeof(float) * (size_t)n_items * d.F);
  w.dpre = take(sizeof(float) * (size_t)n_items * d.F);
  w.wpart = take(sizeof(float) * (size_t)kCnnSplits * 2 * d.n_d * (d.F + 1));
  w.cpart = take(sizeof(float) * (size_t)kCnnConvWg * (d.n_conv * 2 * d.kc * d.kc + d.n_conv));
  w.total = pos;
  return w;
}
}  // namespace

extern "C" {

int64_t fdcnn_param_count(const dpd_fdcnn_desc* desc) {
  CnnDims d;
  return cnn_check(desc, &d) ? d.params : -1;
}

dpd_status fdcnn_workspace_size(const dpd_fdcnn_desc* desc, int64_t n_items, size_t* bytes_host) {
  CnnDims d;
  if (!desc || !bytes_host) return DPD_ERR_NULL;
  if (!cnn_check(desc, &d)) return DPD_ERR_UNSUPPORTED;
  if (n_items < 1 || n_items > ((int64_t)1 << 31) - 1) return DPD_ERR_SHAPE;
  *bytes_host = cnn_ws_layout(d, n_items).total;
  return DPD_OK;
}

dpd_status fdcnn_forward(const dpd_fdcnn_desc* desc, int64_t n_items, const float* s, const float* w,
                         float* out, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  CnnDims d;
  if (!desc || !s || !w || !out || !workspace) return DPD_ERR_NULL;
  if (!cnn_check(desc, &d)) return DPD_ERR_UNSUPPORTED;
  if (n_items < 1 || n_items > ((int64_t)1 << 31) - 1) return DPD_ERR_SHAPE;
  if (!aligned(s, 8) || !aligned(out, 8) || !aligned(w, 4) || !aligned(workspace, 256)) return DPD_ERR_ALIGN;
  if (s == out) return DPD_ERR_SHAPE;
  const CnnWs L = cnn_ws_layout(d, n_items);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  float* h = at<float>(workspace, L.h);
  { DPD_PROF("cnn_conv"); launch_cnn_conv(d, n_items, s, w, h, device_cus(), stream); }
  { DPD_PROF("cnn_out"); launch_cnn_out(d, n_items, h, w, out, stream); }
  return launch_status();
}

dpd_status fdcnn_backward(const dpd_fdcnn_desc* desc, int64_t n_items, const float* s, const float* w,
                          const float* g_out, float* dw, void* workspace, size_t workspace_bytes,
                          hipStream_t stream) {
  CnnDims d;
  if (!desc || !s || !w || !g_out || !dw || !workspace) return DPD_ERR_NULL;
  if (!cnn_check(desc, &d)) return DPD_ERR_UNSUPPORTED;
  if (n_items < 1 || n_items > ((int64_t)1 << 31) - 1) return DPD_ERR_SHAPE;
  if (!aligned(s, 8) || !aligned(g_out, 8) || !aligned(w, 4) || !aligned(dw, 4) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  const CnnWs L = cnn_ws_layout(d, n_items);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  float* h = at<float>(workspace, L.h);
  float* dpre = at<float>(workspace, L.dpre);
  { DPD_PROF("cnn_conv"); launch_cnn_conv(d, n_items, s, w, h, device_cus(), stream); }
  { DPD_PROF("cnn_dh"); launch_cnn_dh(d, n_items, g_out, w, h, dpre, stream); }
  float* wpart = at<float>(workspace, L.wpart);
  { DPD_PROF("cnn_dwout"); launch_cnn_dwout(d, n_items, g_out, h, wpart, stream); }
  { DPD_PROF("cnn_dwout_reduce"); launch_cnn_dwout_reduce(d, wpart, dw, stream); }
  { DPD_PROF("cnn_dwconv"); launch_cnn_dwconv(d, n_items, s, dpre, at<float>(workspace, L.cpart), dw, stream); }
  return launch_status();
}

size_t dpd_acpr_workspace_size(int64_t n, int32_t nfft) {
  if (nfft < 64 || nfft > 4096 || (nfft & (nfft - 1)) || n < nfft) return 0;
  int64_t nseg = (n - nfft) / (nfft / 2) + 1;
  int64_t groups = std::min<int64_t>(nseg, 1024);
  return align_up(sizeof(float) * (size_t)groups * nfft) + align_up(sizeof(float2) * (size_t)kWelchSplits * nfft);
}

dpd_status cascade_acpr(const float* y, int64_t n, int32_t nfft, int32_t half_bins, float* psd,
                        float* acpr, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!y || !psd || !acpr || !workspace) return DPD_ERR_NULL;
  if (nfft < 64 || nfft > 4096 || (nfft & (nfft - 1))) return DPD_ERR_SHAPE;
  if (n < nfft || half_bins < 1 || 3 * half_bins >= nfft / 2) return DPD_ERR_SHAPE;
  if (!aligned(y, 8) || !aligned(psd, 4) || !aligned(acpr, 4) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  size_t need = dpd_acpr_workspace_size(n, nfft);
  if (workspace_bytes < need) return DPD_ERR_WORKSPACE;
  int64_t nseg = (n - nfft) / (nfft / 2) + 1;
  int groups = (int)std::min<int64_t>(nseg, 1024);
  float* seg_part = static_cast<float*>(workspace);
  float2* sums = reinterpret_cast<float2*>(static_cast<char*>(workspace) +
                                           align_up(sizeof(float) * (size_t)groups * nfft));
  { DPD_PROF("welch"); launch_welch(y, n, nfft, seg_part, groups, stream); }
  {
    DPD_PROF("welch_final");
    launch_welch_final(seg_part, groups, (int)nseg, nfft, half_bins, sums, psd, acpr, stream);
  }
  return launch_status();
}

dpd_status dpd_profile_enable(int32_t on) {
  Prof& p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  p.on = on != 0;
  return DPD_OK;
}

int32_t dpd_profile_report(char* buf_host, size_t cap) {
  Prof& p = prof();
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lock(p.mu);
    recs.swap(p.recs);
  }
  std::map<std::string, std::pair<int, double>> acc;
  for (auto& r : recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& e = acc[r.name];
      e.first += 1;
      e.second += ms;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  std::string out;
  for (auto& kv : acc) {
    char line[256];
    snprintf(line, sizeof(line), "%s %d %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  if (buf_host && cap > 0) {
    size_t n = std::min(cap - 1, out.size());
    memcpy(buf_host, out.data(), n);
    buf_host[n] = 0;
  }
  return (int32_t)acc.size();
}

const char* dpd_status_string(dpd_status status) {
  switch (status) {
    case DPD_OK: return "DPD_OK";
    case DPD_ERR_NULL: return "DPD_ERR_NULL: a required pointer is NULL";
    case DPD_ERR_SHAPE: return "DPD_ERR_SHAPE: invalid size, offset table or descriptor";
    case DPD_ERR_UNSUPPORTED: return "DPD_ERR_UNSUPPORTED: request not implemented by this library";
    case DPD_ERR_WORKSPACE: return "DPD_ERR_WORKSPACE: workspace too small";
    case DPD_ERR_LAUNCH: return "DPD_ERR_LAUNCH: the HIP runtime reported an error";
    case DPD_ERR_ALIGN: return "DPD_ERR_ALIGN: misaligned pointer";
    case DPD_ERR_NONFINITE: return "DPD_ERR_NONFINITE: non-finite samples in the NMSE records";
  }
  return "unknown dpd_status";
}

const char* dpd_version(void) { return "dpdmi 0.1 gfx950"; }

}  // extern "C"

// ------------------------------------------------------------------ OFDM downlink
namespace {

bool fdnn_check(const dpd_fdnn_desc* d, NnDims* out) {
  if (!d) return false;
  const NnDims n = nn_dims(d->n_fft, d->users, d->memory, d->hidden, d->n_hidden);
  if (!nn_supported(n)) return false;
  *out = n;
  return true;
}

struct NnWs {
  size_t td = 0, o = 0, part = 0, total = 0;
};
NnWs fdnn_ws_layout(const NnDims& d, int64_t n_sym) {
  NnWs w;
  size_t pos = 0;
  auto take = [&](size_t bytes) { size_t at = pos; pos = align_up(pos + bytes); return at; };
  const size_t row = sizeof(float2) * (size_t)n_sym * d.users * d.n_fft;
  w.td = take(row);
  w.o = take(row);
  w.part = take(sizeof(float) * ((size_t)kFdnnMaxGroups * d.part_floats + d.mid_floats));
  w.total = pos;
  return w;
}

bool fdnn_sym_ok(const NnDims& d, int64_t n_sym) {
  // tile counts (128-sample tiles) stay within int
  return n_sym >= 1 && n_sym * (int64_t)((d.n_fft + 127) / 128) < ((int64_t)1 << 31);
}

bool link_gmp_ok(const dpd_gmp_desc& g, int n_fft) {
  return g.K >= 1 && g.K <= DPD_MAX_GMP_K && g.M >= 0 && g.M <= DPD_MAX_GMP_M && g.L >= 0 &&
         g.L <= DPD_MAX_GMP_L && g.M + g.L < n_fft;
}

dpd_status link_check(const dpd_link_desc* d) {
  if (!d) return DPD_ERR_NULL;
  if (!fft_size_ok(d->n_fft)) return DPD_ERR_SHAPE;
  if (d->n_data < 2 || d->n_data % 2 || d->n_data >= d->n_fft) return DPD_ERR_SHAPE;
  if (d->users < 1 || d->antennas < 1 || d->taps < 1 || d->qam < 4) return DPD_ERR_SHAPE;
  int m = 2;
  while (m * m < d->qam) ++m;
  if (m * m != d->qam) return DPD_ERR_SHAPE;
  if (d->users > 8 || d->antennas > 256 || d->taps > 64 || m > 256) return DPD_ERR_UNSUPPORTED;
  if (!link_gmp_ok(d->pa, d->n_fft)) return DPD_ERR_SHAPE;
  if (d->dpd.K != 0 && !link_gmp_ok(d->dpd, d->n_fft)) return DPD_ERR_SHAPE;
  return DPD_OK;
}

int qam_side(int qam) {
  int m = 2;
  while (m * m < qam) ++m;
  return m;
}

struct LinkWs {
  size_t y = 0, hd = 0, part = 0, total = 0;
};
LinkWs link_ws_layout(const dpd_link_desc& d, int n_sym, int n_ch) {
  LinkWs w;
  size_t pos = 0;
  auto take = [&](size_t bytes) { size_t at = pos; pos = align_up(pos + bytes); return at; };
  w.y = take(sizeof(float2) * (size_t)n_sym * d.antennas * d.n_fft);
  w.hd = take(sizeof(float2) * (size_t)n_ch * d.n_data * d.users * d.antennas);
  w.part = take(sizeof(int32_t) * (size_t)link_rx_parts(d.n_data, n_sym) * d.users);
  w.total = pos;
  return w;
}

bool syms_ok(int32_t n_sym, int32_t spc) { return n_sym >= 1 && spc >= 1; }
int n_channels(int32_t n_sym, int32_t spc) { return (int)((n_sym + (int64_t)spc - 1) / spc); }

}  // namespace

extern "C" {

dpd_status ofdm_fft(int32_t n_fft, int64_t rows, int32_t inverse, const float* in, float* out,
                    hipStream_t stream) {
  if (!in || !out) return DPD_ERR_NULL;
  if (!fft_size_ok(n_fft) || rows < 1 || (inverse != 0 && inverse != 1)) return DPD_ERR_SHAPE;
  if (!aligned(in, 8) || !aligned(out, 8)) return DPD_ERR_ALIGN;
  { DPD_PROF("fft"); launch_fft(in, out, n_fft, rows, inverse != 0, device_cus(), stream); }
  return launch_status();
}

int64_t fdnn_param_count(const dpd_fdnn_desc* desc) {
  NnDims d;
  return fdnn_check(desc, &d) ? d.params : -1;
}

dpd_status fdnn_workspace_size(const dpd_fdnn_desc* desc, int64_t n_sym, size_t* bytes_host) {
  NnDims d;
  if (!desc || !bytes_host) return DPD_ERR_NULL;
  if (!fdnn_check(desc, &d)) return DPD_ERR_UNSUPPORTED;
  if (!fdnn_sym_ok(d, n_sym)) return DPD_ERR_SHAPE;
  *bytes_host = fdnn_ws_layout(d, n_sym).total;
  return DPD_OK;
}

dpd_status fdnn_forward(const dpd_fdnn_desc* desc, int64_t n_sym, const float* s, const float* w,
                        float* out, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  NnDims d;
  if (!desc || !s || !w || !out || !workspace) return DPD_ERR_NULL;
  if (!fdnn_check(desc, &d)) return DPD_ERR_UNSUPPORTED;
  if (!fdnn_sym_ok(d, n_sym)) return DPD_ERR_SHAPE;
  if (!aligned(s, 8) || !aligned(out, 8) || !aligned(w, 4) || !aligned(workspace, 256)) return DPD_ERR_ALIGN;
  const NnWs L = fdnn_ws_layout(d, n_sym);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  float* td = at<float>(workspace, L.td);
  float* o = at<float>(workspace, L.o);
  const int cus = device_cus();
  const int64_t rows = n_sym * d.users;
  { DPD_PROF("fdnn_idft"); launch_fft(s, td, d.n_fft, rows, true, cus, stream); }
  { DPD_PROF("fdnn_net"); launch_fdnn_fwd(d, n_sym, td, w, o, cus, stream); }
  { DPD_PROF("fdnn_dft"); launch_fft(o, out, d.n_fft, rows, false, cus, stream); }
  return launch_status();
}

dpd_status fdnn_backward(const dpd_fdnn_desc* desc, int64_t n_sym, const float* s, const float* w,
                         const float* g_out, float* dw, void* workspace, size_t workspace_bytes,
                         hipStream_t stream) {
  NnDims d;
  if (!desc || !s || !w || !g_out || !dw || !workspace) return DPD_ERR_NULL;
  if (!fdnn_check(desc, &d)) return DPD_ERR_UNSUPPORTED;
  if (!fdnn_sym_ok(d, n_sym)) return DPD_ERR_SHAPE;
  if (!aligned(s, 8) || !aligned(g_out, 8) || !aligned(w, 4) || !aligned(dw, 4) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  const NnWs L = fdnn_ws_layout(d, n_sym);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  float* td = at<float>(workspace, L.td);
  float* gtd = at<float>(workspace, L.o);
  const int cus = device_cus();
  const int64_t rows = n_sym * d.users;
  { DPD_PROF("fdnn_idft"); launch_fft(s, td, d.n_fft, rows, true, cus, stream); }
  // the adjoint of the unitary DFT is the unitary IDFT
  { DPD_PROF("fdnn_idft"); launch_fft(g_out, gtd, d.n_fft, rows, true, cus, stream); }
  float* part = at<float>(workspace, L.part);
  { DPD_PROF("fdnn_bwd"); launch_fdnn_bwd(d, n_sym, td, gtd, w, part, cus, stream); }
  { DPD_PROF("fdnn_reduce"); launch_fdnn_reduce(d, n_sym, part, dw, cus, stream); }
  return launch_status();
}

dpd_status zf_workspace_size(const dpd_link_desc* desc, int32_t n_ch, size_t* bytes_host) {
  if (!desc || !bytes_host) return DPD_ERR_NULL;
  const dpd_status st = link_check(desc);
  if (st != DPD_OK) return st;
  if (n_ch < 1) return DPD_ERR_SHAPE;
  *bytes_host = align_up(sizeof(double) * (size_t)n_ch * desc->n_fft);
  return DPD_OK;
}

dpd_status zf_precoder(const dpd_link_desc* desc, int32_t n_ch, const float* h_est, float p_total,
                       int32_t all_bins, float* pt, float* alpha, void* workspace, size_t workspace_bytes,
                       hipStream_t stream) {
  if (!desc || !h_est || !pt || !alpha || !workspace) return DPD_ERR_NULL;
  const dpd_status st = link_check(desc);
  if (st != DPD_OK) return st;
  if (n_ch < 1 || !(p_total > 0.f) || n_ch > 65535 || (all_bins != 0 && all_bins != 1)) return DPD_ERR_SHAPE;
  if (!aligned(h_est, 8) || !aligned(pt, 8) || !aligned(alpha, 4) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (workspace_bytes < align_up(sizeof(double) * (size_t)n_ch * desc->n_fft)) return DPD_ERR_WORKSPACE;
  {
    DPD_PROF("zf");
    launch_zf(h_est, desc->n_fft, desc->n_data, all_bins, desc->users, desc->antennas, desc->taps, n_ch, p_total,
              pt, at<double>(workspace, 0), alpha, stream);
  }
  return launch_status();
}

dpd_status ofdm_precode(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* pt,
                        const float* alpha, const float* s, int32_t all_bins, float* x, hipStream_t stream) {
  if (!desc || !pt || !alpha || !s || !x) return DPD_ERR_NULL;
  const dpd_status st = link_check(desc);
  if (st != DPD_OK) return st;
  if (!syms_ok(n_sym, sym_per_ch) || n_sym > 65535 || (all_bins != 0 && all_bins != 1)) return DPD_ERR_SHAPE;
  if (!aligned(pt, 8) || !aligned(alpha, 4) || !aligned(s, 8) || !aligned(x, 8)) return DPD_ERR_ALIGN;
  {
    DPD_PROF("precode");
    launch_precode(pt, alpha, s, desc->n_fft, desc->n_data, desc->users, desc->antennas, n_sym, sym_per_ch,
                   all_bins, x, stream);
  }
  return launch_status();
}

dpd_status ofdm_precode_backward(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* pt,
                                 const float* alpha, const float* g_x, int32_t all_bins, float* g_s,
                                 hipStream_t stream) {
  if (!desc || !pt || !alpha || !g_x || !g_s) return DPD_ERR_NULL;
  const dpd_status st = link_check(desc);
  if (st != DPD_OK) return st;
  if (!syms_ok(n_sym, sym_per_ch) || n_sym > 65535 || (all_bins != 0 && all_bins != 1)) return DPD_ERR_SHAPE;
  if (!aligned(pt, 8) || !aligned(alpha, 4) || !aligned(g_x, 8) || !aligned(g_s, 8)) return DPD_ERR_ALIGN;
  {
    DPD_PROF("precode_bwd");
    launch_precode_bwd(pt, alpha, g_x, desc->n_fft, desc->n_data, desc->users, desc->antennas, n_sym, sym_per_ch,
                       all_bins, g_s, stream);
  }
  return launch_status();
}

dpd_status link_workspace_size(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch,
                               size_t* bytes_host) {
  if (!desc || !bytes_host) return DPD_ERR_NULL;
  const dpd_status st = link_check(desc);
  if (st != DPD_OK) return st;
  if (!syms_ok(n_sym, sym_per_ch) || n_sym > 65535) return DPD_ERR_SHAPE;
  *bytes_host = link_ws_layout(*desc, n_sym, n_channels(n_sym, sym_per_ch)).total;
  return DPD_OK;
}

dpd_status ofdm_link(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* x,
                     const float* dpd_coef, const float* pa_coef, float g_re, float g_im, const float* h,
                     const float* alpha, const float* noise, const int32_t* tx, float* r_out, int64_t* errors,
                     void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!desc || !x || !pa_coef || !h || !alpha || !tx || !errors || !workspace) return DPD_ERR_NULL;
  const dpd_status st = link_check(desc);
  if (st != DPD_OK) return st;
  if (desc->dpd.K != 0 && !dpd_coef) return DPD_ERR_NULL;
  if (!syms_ok(n_sym, sym_per_ch) || n_sym > 65535 || !(g_re * g_re + g_im * g_im > 0.f)) return DPD_ERR_SHAPE;
  if (!aligned(x, 8) || !aligned(pa_coef, 8) || !aligned(h, 8) || !aligned(alpha, 4) || !aligned(tx, 4) ||
      !aligned(errors, 8) || !aligned(workspace, 256) || (noise && !aligned(noise, 8)) ||
      (r_out && !aligned(r_out, 8)) || (dpd_coef && !aligned(dpd_coef, 8)))
    return DPD_ERR_ALIGN;
  const int n_ch = n_channels(n_sym, sym_per_ch);
  const LinkWs L = link_ws_layout(*desc, n_sym, n_ch);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  const dpd_link_desc& d = *desc;
  float* y = at<float>(workspace, L.y);
  float* hd = at<float>(workspace, L.hd);
  { DPD_PROF("link_chan"); launch_chan_data(h, d.n_fft, d.n_data, d.users, d.antennas, d.taps, n_ch, hd, stream); }
  {
    DPD_PROF("link_pa");
    launch_link_pa(x, d.n_fft, d.antennas, (int64_t)n_sym * d.antennas, d.dpd.K ? dpd_coef : nullptr,
                   d.dpd.K ? &d.dpd : nullptr, pa_coef, d.pa, y, device_cus(), stream);
  }
  {
    DPD_PROF("link_rx");
    launch_link_rx(y, hd, alpha, g_re, g_im, noise, tx, d.n_fft, d.n_data, d.users, d.antennas, n_sym,
                   sym_per_ch, qam_side(d.qam), r_out, at<int32_t>(workspace, L.part), errors, stream);
  }
  return launch_status();
}

dpd_status ofdm_link_backward(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* x,
                              const float* pa_coef, float g_re, float g_im, const float* h, const float* alpha,
                              const float* g_r, float* g_x, void* workspace, size_t workspace_bytes,
                              hipStream_t stream) {
  if (!desc || !x || !pa_coef || !h || !alpha || !g_r || !g_x || !workspace) return DPD_ERR_NULL;
  const dpd_status st = link_check(desc);
  if (st != DPD_OK) return st;
  if (desc->dpd.K != 0) return DPD_ERR_UNSUPPORTED;
  if (!syms_ok(n_sym, sym_per_ch) || n_sym > 65535 || !(g_re * g_re + g_im * g_im > 0.f)) return DPD_ERR_SHAPE;
  if (!aligned(x, 8) || !aligned(pa_coef, 8) || !aligned(h, 8) || !aligned(alpha, 4) || !aligned(g_r, 8) ||
      !aligned(g_x, 8) || !aligned(workspace, 256))
    return DPD_ERR_ALIGN;
  if (x == g_x) return DPD_ERR_SHAPE;
  const int n_ch = n_channels(n_sym, sym_per_ch);
  const LinkWs L = link_ws_layout(*desc, n_sym, n_ch);
  if (workspace_bytes < L.total) return DPD_ERR_WORKSPACE;
  const dpd_link_desc& d = *desc;
  float* hd = at<float>(workspace, L.hd);
  { DPD_PROF("link_chan"); launch_chan_data(h, d.n_fft, d.n_data, d.users, d.antennas, d.taps, n_ch, hd, stream); }
  float* g_y = at<float>(workspace, L.y);
  {
    DPD_PROF("link_rx_bwd");
    launch_link_rx_bwd(hd, alpha, g_re, g_im, g_r, d.n_fft, d.n_data, d.users, d.antennas, n_sym, sym_per_ch, g_y,
                       stream);
  }
  { DPD_PROF("link_pa_bwd"); launch_link_pa_bwd(x, g_y, d.n_fft, d.antennas, n_sym, pa_coef, d.pa, g_x, device_cus(), stream); }
  return launch_status();
}

}  // extern "C"
