/*
 * dpdmi — TDNN digital predistorter cascaded with a GMP power-amplifier model,
 * forward, NMSE and hand-written backward on AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2205.05158 (Wu, Gustavsson, Valkama, Graell i Amat, Wymeersch,
 * "Frequency-domain digital predistortion for Massive MU-MIMO-OFDM Downlink").
 *   - DPD: the time-domain DPD of eq. (8), u[n] = f_theta(x[n], ..., x[n-T+1]),
 *     realised as the tapped-delay-line network of Sec. III-C: per tap the
 *     features (Re, Im, |x|, |x|^2, |x|^3), fully connected tanh hidden layers,
 *     two linear outputs (Re u, Im u).
 *   - PA: the PA with memory of eq. (7), instantiated by the GMP of eq. (9)
 *     (this header's K, M, L are the paper's K, L3, G).
 *   - Target: the linear PA of Sec. II-B, y[n] = G x[n];  NMSE = sum|y-Gx|^2 / sum|Gx|^2.
 *   - Training: MSE through the differentiable chain (Sec. V-A-2); the loss here
 *     is the linear NMSE pooled over the streams that share one parameter set.
 *
 * Conventions for every entry point
 *   - Pointers named *_host are host memory; every other array pointer is DEVICE
 *     memory.  The caller allocates and owns every buffer, including the
 *     workspace.  The library never allocates device memory, never synchronises
 *     the device, and enqueues all work on the caller's `stream` (in order); the
 *     one exception is dpd_autotune, which waits for its own timing events.
 *   - Complex sample streams are interleaved float32 (re, im), 8 bytes per sample,
 *     8-byte aligned.  Streams are concatenated; stream s occupies samples
 *     [offsets_host[s], offsets_host[s+1]).  Each stream is independent and
 *     zero-padded on both ends (no state crosses a stream boundary).
 *   - Arguments are validated on the host before any HIP call; on failure a
 *     negative dpd_status is returned and nothing is enqueued.  A launch failure
 *     reported by the runtime after enqueueing returns DPD_ERR_LAUNCH.
 *   - Calls are thread-safe; the library's only mutable global state is a lazily
 *     filled, mutex-guarded cache of device properties, the launch-shape table
 *     (dpd_tune_set / dpd_autotune) and the opt-in kernel timer
 *     (dpd_profile_enable), each mutex-guarded.
 */
#ifndef DPDMI_H
#define DPDMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hipStream_t;

typedef enum {
    DPD_OK = 0,
    DPD_ERR_NULL = -1,         /* a required pointer is NULL                          */
    DPD_ERR_SHAPE = -2,        /* a size, offset table or descriptor value is invalid */
    DPD_ERR_UNSUPPORTED = -3,  /* valid request the library does not implement      */
    DPD_ERR_WORKSPACE = -4,    /* workspace smaller than dpd_workspace_size() says    */
    DPD_ERR_LAUNCH = -5,       /* the HIP runtime reported an error                   */
    DPD_ERR_ALIGN = -6,        /* a pointer is not aligned as documented              */
    DPD_ERR_NONFINITE = -7     /* an NMSE record reports non-finite samples
                                  (dpd_nmse_status, on host copies of the records)    */
} dpd_status;

typedef enum { DPD_FP32 = 0, DPD_BF16 = 1 } dpd_precision;
typedef enum { DPD_IMPL_TUNED = 0, DPD_IMPL_PLAIN = 1 } dpd_impl;

enum { DPD_MAX_STREAMS = 128, DPD_MAX_TAPS = 32, DPD_MAX_HIDDEN = 256, DPD_MAX_LAYERS = 8,
       DPD_MAX_GMP_K = 12, DPD_MAX_GMP_M = 15, DPD_MAX_GMP_L = 8 };

/* TDNN DPD (eq. (8) slot, Sec. III-C network).  Features of tap t (t = 0..T-1) of
 * sample n are (Re z, Im z, |z|, |z|^2, |z|^3) with z = x[n-t] (0 before the
 * stream start), at input index 5t+j.  h_0 = features, h_i = tanh(W_i h_{i-1} + b_i),
 * (o0, o1) = W_o h_nl + b_o, u = o0 + j o1 (+ x[n] if residual).
 * Packed float32 weights (P = dpd_tdnn_param_count): W1[H][5T] b1[H]
 * (W_i[H][H] b_i[H]) for i = 2..nl, W_o[2][H] b_o[2]; rows are output neurons.
 * DPD_IMPL_TUNED runs every shape with T <= 32, H <= 128 and nl <= 4: the paper's three
 * sizes (T, nl, H) = (4, 2, 20), (10, 3, 64), (16, 4, 128) on kernels compiled for them,
 * the others on generic instantiations compiled for T rounded up to 8, 16 or 32 and H to
 * 32, 64 or 128 (zero-padded weights, padding taps masked); larger shapes return
 * DPD_ERR_UNSUPPORTED there (DPD_IMPL_PLAIN, float32, takes every valid shape). */
typedef struct {
    int32_t taps;       /* T, 1..DPD_MAX_TAPS                               */
    int32_t n_hidden;   /* nl, 1..DPD_MAX_LAYERS                            */
    int32_t hidden;     /* H, 1..DPD_MAX_HIDDEN                             */
    int32_t residual;   /* 0 or 1                                           */
    int32_t precision;  /* dpd_precision: arithmetic of the hidden layers   */
    int32_t impl;       /* dpd_impl: tuned MFMA kernels or plain kernels    */
} dpd_tdnn_desc;

/* GMP PA, eq. (9): y[n] = sum_{k=0}^{K-1} sum_{l=0}^{M} a_{k,l} u[n-l] |u[n-l]|^k
 *   + sum_{k=1}^{K-1} sum_{l=0}^{M} sum_{g=1}^{L} ( b_{k,l,g} u[n-l] |u[n-l-g]|^k
 *                                                 + c_{k,l,g} u[n-l] |u[n-l+g]|^k ),
 * u = 0 outside the stream.  Packed complex float32 coefficients
 * (J = dpd_gmp_coeff_count): a[K][M+1], b[K-1][M+1][L], c[K-1][M+1][L],
 * b and c indexed from k = 1 and g = 1.  The tuned gradient path (dpd_backward,
 * dpd_cascade with dW, dpd_autotune) takes K <= 9, M <= 7, L <= 4: the orders (5, 3, 2),
 * (7, 5, 3), (9, 7, 4) and (7, 3, 1) on kernels compiled for them, the others on the
 * (9, 7, 4) kernels with zero-padded coefficients (their reverse-mode table, and so the
 * workspace, then has that order's size); larger orders return DPD_ERR_UNSUPPORTED there
 * (DPD_IMPL_PLAIN takes every valid order). */
typedef struct {
    int32_t K;          /* nonlinear order, 1..DPD_MAX_GMP_K   */
    int32_t M;          /* memory depth (paper L3), 0..DPD_MAX_GMP_M */
    int32_t L;          /* cross-term length (paper G), 0..DPD_MAX_GMP_L */
} dpd_gmp_desc;

/* A batch of independent streams.  per_stream_params = 0: every stream uses the
 * one parameter set (weights w, coefficients coef);  = 1: stream s uses set s,
 * i.e. w + s*P and coef + s*2J.  The number of parameter sets is S or 1. */
typedef struct {
    int32_t n_streams;           /* S, 1..DPD_MAX_STREAMS                          */
    int32_t per_stream_params;   /* 0 or 1                                         */
    const int64_t* offsets_host; /* [S+1], offsets[0] = 0, strictly increasing     */
} dpd_batch;

/* Parameter counts (< 0 on an invalid descriptor). */
int64_t dpd_tdnn_param_count(const dpd_tdnn_desc* tdnn);
int64_t dpd_gmp_coeff_count(const dpd_gmp_desc* gmp);

/* Bytes of device workspace every call below needs for this problem (an upper
 * bound over the launch shapes the library may choose).  The same workspace may
 * be reused by consecutive calls on one stream; concurrent calls need their own.
 * Tuned BF16 models include the forward's stored hidden activations, which the
 * reverse mode reads instead of recomputing them: n_hidden x padded width x 2 bytes
 * per sample (1 KB per sample for 4 layers of 128; 17 GB for 2^24 samples). */
dpd_status dpd_workspace_size(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp,
                              const dpd_batch* batch, size_t* bytes_host);

/* DPD forward (eq. (8)): x [n_total][2] -> u [n_total][2]. */
dpd_status dpd_forward(const dpd_tdnn_desc* tdnn, const dpd_batch* batch,
                       const float* x, const float* w, float* u,
                       void* workspace, size_t workspace_bytes, hipStream_t stream);

/* GMP PA forward (eq. (9)): u [n_total][2] -> y [n_total][2].  u and y must not overlap. */
dpd_status pa_gmp_forward(const dpd_gmp_desc* gmp, const dpd_batch* batch,
                          const float* u, const float* coef, float* y, hipStream_t stream);

/* NMSE records.  The NMSE of y against the linear target G x (Sec. II-B) is reported
 * as one record of DPD_NMSE_FIELDS floats per stream plus one pooled over all streams:
 *   (E, R, NMSE_dB, n_nonfinite),  E = sum|y-Gx|^2, R = sum|Gx|^2, NMSE_dB = 10 log10(E/R),
 * accumulated in float32 with compensated (Neumaier) sums.  n_nonfinite counts the
 * samples whose |y-Gx|^2 or |Gx|^2 is not a finite float32 (NaN or infinite inputs or
 * outputs, or squares beyond the float32 range); such samples still enter E and R, so
 * E, NMSE_dB and the loss of their stream and parameter set are then not finite.  The
 * count is exact below 2^24 samples per record.  Records are written on the device
 * without synchronising; dpd_nmse_status checks host copies of them. */
enum { DPD_NMSE_FIELDS = 4 };

/* Host only, no HIP call: DPD_ERR_NONFINITE if any of the n_records records at
 * nmse_host (host float[n_records][DPD_NMSE_FIELDS]) has n_nonfinite > 0, a non-finite
 * E or R, or an NMSE_dB that is NaN or +inf (-inf, the exact match E = 0, is accepted);
 * DPD_OK otherwise; DPD_ERR_NULL / DPD_ERR_SHAPE for a null pointer or n_records < 1. */
dpd_status dpd_nmse_status(const float* nmse_host, int64_t n_records);

/* NMSE of y against the linear target G x (Sec. II-B), per stream and pooled.
 * out: device float[(S+1)][DPD_NMSE_FIELDS]: record s < S of stream s, record S
 * pooled over all streams. */
dpd_status cascade_nmse(const dpd_batch* batch, const float* y, const float* x,
                        float g_re, float g_im, float* out,
                        void* workspace, size_t workspace_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): cascade_nmse without a workspace.
 * Same arguments, records and kernels as cascade_nmse; the partial sums (one record per
 * tile of 256 samples, a tile count per stream rounded up, plus one per 256 tiles of
 * each stream for the final pass) live in a static device array of
 * DPD_NOALLOC_NMSE_MAX_TILES records of 16 bytes (4 MiB, up to about 2^26 samples), held
 * by each device the library runs on until the process ends.  A problem needing more
 * records returns DPD_ERR_WORKSPACE before any HIP call.  The call allocates
 * nothing and calls no allocating routine; the array's device address is looked up once
 * per device (hipGetSymbolAddress, the device current) on the first call there.  Every
 * call on one device shares the array: calls that may overlap on one device (other
 * streams or host threads) race and must be serialised by the caller; the array keeps
 * the last call's partials, and each call writes every partial it reads, so nothing
 * needs clearing. */
enum { DPD_NOALLOC_NMSE_MAX_TILES = 1 << 18 };
dpd_status cascade_nmse_noalloc(const dpd_batch* batch, const float* y, const float* x,
                                float g_re, float g_im, float* out, hipStream_t stream);

/* Direct-learning gradient (Sec. V-A-2): runs DPD -> GMP -> NMSE and the reverse
 * mode through both, returning for each parameter set p the pooled loss
 * loss[p] = sum_{s in p} E_s / sum_{s in p} R_s and dw[p] = d loss[p] / d w_p
 * (same packed layout as w).  loss: device float[n_sets]; dw: device float[n_sets*P].
 * d|u|/du is taken as 0 at u = 0.  Deterministic: identical inputs give bitwise
 * identical results for a given launch shape.  A set whose streams hold non-finite
 * samples (see the NMSE records) gets a non-finite loss and dw; other sets are not
 * affected. */
dpd_status dpd_backward(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp,
                        const dpd_batch* batch, const float* x, const float* w,
                        const float* coef, float g_re, float g_im, float* dw, float* loss,
                        void* workspace, size_t workspace_bytes, hipStream_t stream);

/* The whole cascade in one call: optional u and y outputs (NULL to skip),
 * NMSE records as cascade_nmse (nmse: device float[(S+1)][DPD_NMSE_FIELDS], may be
 * NULL), and when dw is non-NULL the gradient and pooled loss as dpd_backward
 * (loss required with dw). */
dpd_status dpd_cascade(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp,
                       const dpd_batch* batch, const float* x, const float* w,
                       const float* coef, float g_re, float g_im,
                       float* u, float* y, float* nmse, float* dw, float* loss,
                       void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Ideal linear-clipping PA, the minimum-distortion reference PA of the paper's SER
 * comparison (Sec. V-B-2): unit gain up to the clipping level, constant envelope beyond
 * it, phase kept, no memory:
 *   y[n] = u[n]                          if |u[n]| <= a_clip,
 *   y[n] = a_clip u[n] / |u[n]|          otherwise.
 * u, y: device float[n][2], 8-byte aligned; y may equal u (in place).  a_clip finite
 * and > 0, n >= 1 (DPD_ERR_SHAPE otherwise).  |u| is formed without overflow for every
 * finite u; a NaN sample stays NaN, an infinite one becomes NaN. */
dpd_status pa_clip_forward(int64_t n, const float* u, float a_clip, float* y, hipStream_t stream);

/* The cascade DPD -> linear-clipping PA -> NMSE: dpd_cascade with the clipping PA above
 * in place of the GMP PA.  Same outputs (u, y, NMSE records, and with dw the pooled loss
 * per parameter set and its gradient), same argument rules; the workspace is
 * dpd_workspace_size(tdnn, NULL, batch).  Reverse mode of the PA: g_u = g_y below the
 * clip; beyond it only the phase of u moves y, g_u = (a_clip / |u|)(g_y - v Re(conj(v)
 * g_y)) with v = u / |u|; at |u| = a_clip exactly the linear branch's derivative is
 * taken. */
dpd_status dpd_cascade_clip(const dpd_tdnn_desc* tdnn, const dpd_batch* batch, const float* x,
                            const float* w, float a_clip, float g_re, float g_im,
                            float* u, float* y, float* nmse, float* dw, float* loss,
                            void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Launch shapes of the tuned path.  The many-stream persistent launches (the
 * per-antenna DPDs of the paper's massive-MIMO setting, Sec. II and V) run with
 * tile shapes and grid sizes picked at run time among compiled variants:
 *   fwd_waves      waves per forward workgroup: 8, 12 or 16 (tile = waves x 16 samples
 *                  in bf16, waves x 32 in fp32);
 *   fwd_wg_per_cu  forward workgroups per compute unit, 1..4 (capped by the tiles);
 *   bwd_wg_per_cu  backward (reverse-mode) workgroups per compute unit, 1..2
 *                  (capped at 512 workgroups and by the tiles);
 *   gmp_tile       samples per GMP reverse-mode workgroup: 256 or 512.
 * The shape never changes u or y (bitwise); the NMSE, the loss and dW may change by
 * float32 rounding (their partial sums are grouped by tile and workgroup).
 * A problem is keyed by the TDNN descriptor, the GMP descriptor (none for
 * dpd_forward) and the batch signature (n_streams, per_stream_params, total and
 * longest stream length).  Problems without an entry use the defaults. */
typedef struct {
    int32_t fwd_waves;
    int32_t fwd_wg_per_cu;
    int32_t bwd_wg_per_cu;
    int32_t gmp_tile;
} dpd_tune;

/* Shape the tuned-path calls use for this problem (its table entry, else the
 * defaults).  gmp may be NULL (the dpd_forward key).  Host only; no HIP call.
 * DPD_ERR_UNSUPPORTED for the plain implementation. */
dpd_status dpd_tune_get(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp,
                        const dpd_batch* batch, dpd_tune* out_host);

/* Install (tune_host != NULL, validated against the ranges above: DPD_ERR_SHAPE
 * otherwise) or remove (tune_host == NULL) this problem's table entry.  Host only. */
dpd_status dpd_tune_set(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp,
                        const dpd_batch* batch, const dpd_tune* tune_host);

/* Autotuner: on the given inputs, times reps (1..1000) back-to-back launches of every
 * candidate shape of each kernel (12 forward shapes, 2 GMP tiles, 2 backward grids;
 * the kernels run one after another, so each is tuned on its own), installs the
 * fastest combination as this problem's entry (gmp key = gmp) and returns it.  It
 * enqueues that work on `stream`, records HIP events on it and waits for them (it
 * blocks; not for the hot loop), and writes only workspace memory.  Tuned
 * implementation with GMP orders of the tuned gradient path only (else
 * DPD_ERR_UNSUPPORTED). */
dpd_status dpd_autotune(const dpd_tdnn_desc* tdnn, const dpd_gmp_desc* gmp,
                        const dpd_batch* batch, const float* x, const float* w,
                        const float* coef, float g_re, float g_im, int32_t reps,
                        void* workspace, size_t workspace_bytes, hipStream_t stream,
                        dpd_tune* out_host);

/* Mean squared error of complex symbols: the supervised criterion the paper trains its
 * frequency-domain DPDs with (Sec. V-A-2), for n complex values z_i (e.g. equalised
 * received symbols) against targets t_i (the transmitted symbols):
 *   loss = sum_i |z_i - t_i|^2 / n,  grad_i = 2 (z_i - t_i) / n  (= dloss/dRe + j dloss/dIm),
 * summed in float32 with compensated sums in a fixed order (deterministic).
 * z, t: device float[n][2]; out: device float[2] = (loss, count of i whose |z_i - t_i|^2
 * is not finite); grad: device float[n][2] (not aliasing z or t) or NULL.  The
 * workspace (dpd_symbol_mse_workspace_size) holds per-tile partial sums. */
dpd_status dpd_symbol_mse_workspace_size(int64_t n, size_t* bytes_host);
dpd_status dpd_symbol_mse(int64_t n, const float* z, const float* t, float* out, float* grad,
                          void* workspace, size_t workspace_bytes, hipStream_t stream);

/* One Adam step on n float32 parameters in place: the optimiser the paper trains its
 * DPD networks with (Sec. V-A-2, learning rate 0.001), with the update rule of
 * Kingma & Ba (Algorithm 1):
 *   m = beta1 m + (1 - beta1) g;   v = beta2 v + (1 - beta2) g^2;
 *   w -= lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps).
 * grad, w, m, v: device float[n], 4-byte aligned (16-byte aligned buffers take the
 * vector path), pairwise non-overlapping (DPD_ERR_SHAPE otherwise).  m and v hold the
 * optimiser state between calls (zero before step 1, owned by the caller).  step >= 1
 * is the caller's step counter (the bias corrections use it); 0 <= beta1, beta2 < 1;
 * lr finite; eps finite and >= 0.  The hyper-parameters are double so that 1 - beta
 * is formed before rounding to the float32 the kernel computes in.  With grad = the
 * dw of dpd_backward (all parameter sets concatenated) this is one direct-learning
 * update. */
dpd_status dpd_adam_step(const float* grad, float* w, float* m, float* v, int64_t n,
                         int32_t step, double lr, double beta1, double beta2, double eps,
                         hipStream_t stream);

/* Least-squares fit of a GMP DPD by indirect learning: the TD-GMP benchmark of the
 * paper (the per-antenna DPD with the monomials of eq. (9), coefficients found by
 * mean-square-error estimation, Sec. III-B) identified as a post-inverse at the PA output
 * (least squares between the post-distorter output and the PA input, Sec. V-A-2).
 * For every parameter set p (per stream, or one pooled over all streams):
 *   z = y / G,  Phi = the eq. (9) monomials of z (flat coefficient order a, b, c; zero
 *   padding at both ends of every stream),
 *   (Phi^H Phi + lambda I) c = Phi^H t,  lambda = ridge * trace(Phi^H Phi) / J,
 * the normal equations accumulated in float64 on the matrix cores and solved by a
 * complex Cholesky factorisation in float64.
 * y, t: device float[n_total][2] (PA output and PA input); coef: device float[n_sets][J][2]
 * (usable directly as pa_gmp_forward coefficients of the DPD); info: device
 * int32[n_sets], 0 on success, k + 1 if pivot k of the factorisation is not positive
 * (rank-deficient basis, e.g. a stream shorter than J samples with ridge = 0; coef of
 * that set is then zero).  normal_out (may be NULL): device double[n_sets][J][J+1][2], the
 * rows of [Phi^H Phi | Phi^H t] (16-byte aligned).  ridge finite and >= 0.  Supported
 * for J <= 1024.  The workspace (gmp_ls_workspace_size) holds per-split partial Gram
 * blocks and the factorisation. */
dpd_status gmp_ls_workspace_size(const dpd_gmp_desc* gmp, const dpd_batch* batch,
                                 size_t* bytes_host);
dpd_status gmp_ls_fit(const dpd_gmp_desc* gmp, const dpd_batch* batch, const float* y,
                      float g_re, float g_im, const float* t, double ridge, float* coef,
                      int32_t* info, double* normal_out, void* workspace,
                      size_t workspace_bytes, hipStream_t stream);

/* FD-CNN DPD, the paper's proposed frequency-domain network (Sec. IV-A; Sec. V-A uses
 * n_d = 384 data subcarriers, side = 20, n_conv = 2, kc = 3, ReLU), applied to a batch of
 * n_items UE symbol vectors (one UE's N_d data-subcarrier symbols of one OFDM symbol):
 * the vector fills a side x side grid row-major (zero padded); its Re and Im planes
 * are convolved by n_conv kernels kc x kc (each spanning both planes, biased, zero
 * padding keeping the plane size), ReLU, flattened plane-major (F = n_conv side^2) and
 * mapped by a linear layer with bias to 2 n_d outputs: Re of the predistorted symbols,
 * then Im.  Parameters w (float): conv weights [n_conv][2][kc][kc], conv biases
 * [n_conv], output weights [2 n_d][F], output biases [2 n_d].
 * Supported: side <= 32, n_d <= side^2, n_conv <= 4, kc odd <= 7. */
typedef struct {
    int32_t n_d;      /* data subcarriers per symbol vector */
    int32_t side;     /* grid side, side^2 >= n_d (the paper: ceil(sqrt(n_d))) */
    int32_t n_conv;   /* convolution kernels */
    int32_t kc;       /* kernel size (odd) */
} dpd_fdcnn_desc;

/* Parameter count (< 0 for an invalid or unsupported descriptor). */
int64_t fdcnn_param_count(const dpd_fdcnn_desc* desc);
dpd_status fdcnn_workspace_size(const dpd_fdcnn_desc* desc, int64_t n_items, size_t* bytes_host);
/* s: device float[n_items][n_d][2]; out: device float[n_items][n_d][2] (may not alias s). */
dpd_status fdcnn_forward(const dpd_fdcnn_desc* desc, int64_t n_items, const float* s,
                         const float* w, float* out, void* workspace, size_t workspace_bytes,
                         hipStream_t stream);
/* Reverse mode for the real-convention output gradient g_out = dL/dRe + j dL/dIm
 * (device float[n_items][n_d][2]): dw (device float[param count], packed like w) =
 * dL/dw summed over the items (fixed summation order: deterministic). */
dpd_status fdcnn_backward(const dpd_fdcnn_desc* desc, int64_t n_items, const float* s,
                          const float* w, const float* g_out, float* dw, void* workspace,
                          size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------ OFDM downlink
 * Multi-user OFDM downlink around the frequency-domain DPDs (Sec. II-A, Sec. III-C):
 * N = n_fft subcarriers; n_data of them carry data, on subcarriers 1..n_data/2 and
 * N - n_data/2..N - 1 (data symbol d on 1 + d for d < n_data/2, else N - n_data + d),
 * the rest (DC, outer band) are guard; U users, B antennas, T channel taps.  Every delay
 * inside an OFDM symbol is cyclic (index mod N): the frequency-domain channel of
 * eq. (5) holds exactly only for a cyclic convolution, i.e. a cyclic prefix longer than
 * every memory.  Complex arrays are interleaved float [..][2]; all pointers device
 * pointers, 8-byte aligned for complex arrays, workspaces 256-byte aligned. */

/* Batched unitary DFT over `rows` contiguous rows of n_fft points, n_fft a power of two
 * in [2, 4096]: inverse = 0 gives X_k = N^-1/2 sum_n x_n e^{-2 pi i kn/N}, inverse = 1
 * the IDFT of eq. (2) (+i, same scale).  in may equal out. */
dpd_status ofdm_fft(int32_t n_fft, int64_t rows, int32_t inverse, const float* in, float* out,
                    hipStream_t stream);

/* FD-NN DPD (Sec. III-C): each UE's subcarrier vector to the time domain (unitary IDFT),
 * delay lines of memory + 1 samples of all U UEs as 2 U (memory + 1) real inputs (input
 * 2 (u (memory + 1) + t) + {0, 1} = Re, Im of UE u's sample n - t), n_hidden fully
 * connected ReLU layers of `hidden` neurons, 2 U linear outputs (2u = Re, 2u + 1 = Im of
 * UE u) and a unitary DFT per UE back to all N subcarriers (guard subcarriers included).
 * Parameters w (float): W1[hidden][2 U (memory+1)] b1[hidden] (W_i[hidden][hidden]
 * b_i[hidden])_{i=2..n_hidden} Wo[2U][hidden] bo[2U].
 * Supported: users <= 8, memory <= 7, 2 users (memory + 1) <= 64, hidden <= 32,
 * n_hidden 1 or 2, n_fft as ofdm_fft. */
typedef struct {
    int32_t n_fft;     /* N */
    int32_t users;     /* U */
    int32_t memory;    /* delay-line memory (the paper's L4) */
    int32_t hidden;    /* D */
    int32_t n_hidden;  /* K^NN */
} dpd_fdnn_desc;

/* Parameter count (< 0 for an invalid or unsupported descriptor). */
int64_t fdnn_param_count(const dpd_fdnn_desc* desc);
dpd_status fdnn_workspace_size(const dpd_fdnn_desc* desc, int64_t n_sym, size_t* bytes_host);
/* s, out: float[n_sym][U][N][2] (UE symbol vectors on the subcarriers; out may equal s). */
dpd_status fdnn_forward(const dpd_fdnn_desc* desc, int64_t n_sym, const float* s, const float* w,
                        float* out, void* workspace, size_t workspace_bytes, hipStream_t stream);
/* Reverse mode for the real-convention output gradient g_out = dL/dRe + j dL/dIm
 * (float[n_sym][U][N][2]): dw (float[param count], packed like w) = dL/dw summed over
 * every symbol, UE and sample (fixed summation order: deterministic). */
dpd_status fdnn_backward(const dpd_fdnn_desc* desc, int64_t n_sym, const float* s, const float* w,
                         const float* g_out, float* dw, void* workspace, size_t workspace_bytes,
                         hipStream_t stream);

/* Downlink link.  Channel taps h: float[n_ch][T][U][B][2].  OFDM symbol i uses channel
 * realisation i / sym_per_ch (n_ch = ceil(n_sym / sym_per_ch)).
 * Supported: users <= 8, antennas <= 256, taps <= 64, qam = m^2 with 2 <= m <= 256, PA
 * and DPD GMP orders within the DPD_MAX_GMP_* ranges with M + L < n_fft, 2 <= n_data <
 * n_fft even. */
typedef struct {
    int32_t n_fft, n_data, users, antennas, taps, qam;
    dpd_gmp_desc pa;    /* per-antenna PA model, eq. (9) with cyclic delays */
    dpd_gmp_desc dpd;   /* per-antenna TD-GMP DPD in front of the PA; dpd.K = 0: none */
} dpd_link_desc;

dpd_status zf_workspace_size(const dpd_link_desc* desc, int32_t n_ch, size_t* bytes_host);
/* ZF precoding (eq. (6)) from the estimated taps h_est: pt[c][k] = H_k^H (H_k H_k^H)^-1
 * (float[n_ch][N][B][U][2]), H_k = sum_t H_t e^{-2 pi i k t / N}, computed in FP64
 * (H_k H_k^H must be nonsingular), on the data subcarriers (all_bins = 0; the guard
 * entries of pt are not written) or on every subcarrier (all_bins = 1, for guard-band
 * precoding); alpha[c] (float[n_ch]) = sqrt(p_total / mean over the data subcarriers of
 * tr(pt^H pt)), so that the precoder alpha pt meets the average transmit power p_total
 * with unit-energy symbols (one alpha per channel realisation). */
dpd_status zf_precoder(const dpd_link_desc* desc, int32_t n_ch, const float* h_est, float p_total,
                       int32_t all_bins, float* pt, float* alpha, void* workspace, size_t workspace_bytes,
                       hipStream_t stream);
/* x[i][b][k] = alpha[c] sum_u pt[c][k][b][u] s[i][u][k] (eq. (1)) on the data subcarriers
 * (all_bins = 0) or on every subcarrier (all_bins = 1: the guard-band precoding an FD-NN
 * output needs), 0 elsewhere.  s: float[n_sym][U][N][2]; x: float[n_sym][B][N][2]; pt and
 * alpha hold (at least) the ceil(n_sym / sym_per_ch) realisations the symbols use. */
dpd_status ofdm_precode(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* pt,
                        const float* alpha, const float* s, int32_t all_bins, float* x,
                        hipStream_t stream);
dpd_status link_workspace_size(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch,
                               size_t* bytes_host);
/* The precoded x (float[n_sym][B][N][2]) through, per antenna b: unitary IDFT (eq. (2)),
 * the optional TD-GMP DPD (dpd_coef float[B][Jd][2]), the PA (pa_coef float[B][J][2],
 * eq. (7)), unitary DFT; then per data subcarrier the true channel h (eq. (5)) plus the
 * frequency-domain noise (float[n_sym][U][N][2], or NULL for none), equalised by
 * 1 / (alpha[c] G) with G = g_re + j g_im the PA's linear gain, and decided to the
 * nearest unit-energy square-QAM point, index i_re m + i_im of the point
 * ((2 i_re - m + 1) + j (2 i_im - m + 1)) / sqrt(2 (m^2 - 1) / 3).  tx: int32
 * [n_sym][U][n_data] transmitted indices; r_out (NULL or float[n_sym][U][n_data][2]) the
 * equalised symbols; errors: int64[U] symbol errors per UE (overwritten).  h and alpha
 * hold (at least) ceil(n_sym / sym_per_ch) realisations. */
dpd_status ofdm_link(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* x,
                     const float* dpd_coef, const float* pa_coef, float g_re, float g_im,
                     const float* h, const float* alpha, const float* noise, const int32_t* tx,
                     float* r_out, int64_t* errors, void* workspace, size_t workspace_bytes,
                     hipStream_t stream);

/* Reverse mode of the link for a real loss on the equalised symbols (receiver-side
 * training, Sec. V-A-2): given g_r = dL/dRe + j dL/dIm of r_out (float[n_sym][U][n_data][2]),
 * g_x (float[n_sym][B][N][2], not aliasing x) = the gradient with respect to the precoded
 * x of ofdm_link: the adjoints of equalisation and channel, of the DFT (the IDFT), of the
 * PA (eq. (9) differentiated, cyclic delays, d|u|/du = 0 at u = 0) and of the IDFT (the
 * DFT).  Decisions and noise do not enter; desc.dpd.K must be 0 (DPD_ERR_UNSUPPORTED
 * otherwise).  Workspace as link_workspace_size. */
dpd_status ofdm_link_backward(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* x,
                              const float* pa_coef, float g_re, float g_im, const float* h, const float* alpha,
                              const float* g_r, float* g_x, void* workspace, size_t workspace_bytes,
                              hipStream_t stream);
/* Adjoint of ofdm_precode: g_s[i][u][k] = alpha[c] sum_b conj(pt[c][k][b][u]) g_x[i][b][k]
 * on the precoded subcarriers (as all_bins), 0 elsewhere; g_s float[n_sym][U][N][2]. */
dpd_status ofdm_precode_backward(const dpd_link_desc* desc, int32_t n_sym, int32_t sym_per_ch, const float* pt,
                                 const float* alpha, const float* g_x, int32_t all_bins, float* g_s,
                                 hipStream_t stream);

/* Welch PSD of one stream y [n][2] (nfft-point segments, periodic Hann window,
 * 50 % overlap, no detrending, scaled by 1/sum(w^2)), bins in natural FFT order,
 * and the ACPR with main channel |k| <= half_bins, adjacent channels
 * half_bins < |k| <= 3 half_bins.  nfft is a power of two in [64, 4096];
 * n >= nfft; 3*half_bins < nfft/2.  psd: device float[nfft];
 * acpr: device float[3] = (ACPR_L dB, ACPR_U dB, max). */
dpd_status cascade_acpr(const float* y, int64_t n, int32_t nfft, int32_t half_bins,
                        float* psd, float* acpr, void* workspace, size_t workspace_bytes,
                        hipStream_t stream);
size_t dpd_acpr_workspace_size(int64_t n, int32_t nfft);

/* Opt-in kernel timing, for profiling tools.  While enabled (on != 0), every kernel
 * the library launches is bracketed by two HIP events recorded on the caller's
 * stream (the only case in which the library creates runtime objects).
 * dpd_profile_report waits for the recorded events, writes one line
 * "<kernel> <launches> <total ms>" per kernel into buf_host (NUL-terminated,
 * truncated to cap bytes), releases the events and returns the number of kernels. */
dpd_status dpd_profile_enable(int32_t on);
int32_t dpd_profile_report(char* buf_host, size_t cap);

/* Human-readable name of a status code (static storage). */
const char* dpd_status_string(dpd_status status);

/* Library build identification (static storage). */
const char* dpd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DPDMI_H */
