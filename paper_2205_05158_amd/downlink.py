"""Multi-user OFDM downlink on the device (Sec. II-A, Sec. III-C): the FD-NN DPD and the
ZF-precoded link with per-antenna PAs, channel, noise and QAM decisions, their reverse
modes, and the receiver-side training of the frequency-domain DPDs (Sec. V-A-2).

`FdNn` holds the FD-NN descriptor and a workspace sized for a maximum number of OFDM
symbols; `FdNnFn` makes its output a torch.autograd.Function of the packed weights.
`Downlink` holds a link descriptor and runs ZF precoding, precoding, the link (the
symbol error count per UE) and the adjoints of the last two.  `receiver_loss_grad*` and
`train_receiver` compose them into the supervised criterion and its Adam loop.  All
arrays are contiguous float32 device tensors with a trailing (re, im) axis, except the
int32 transmitted QAM indices.
"""
from __future__ import annotations

import torch

from . import _lib as L


def _check_c(t, shape, name):
    if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected contiguous float32 {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


class FdNn:
    def __init__(self, n_fft=4096, users=8, memory=3, hidden=15, n_hidden=1, max_sym=1, device="cuda"):
        self.desc = L.fdnn_desc(n_fft, users, memory, hidden, n_hidden)
        self.P = L.fdnn_param_count(self.desc)
        if self.P < 0:
            raise RuntimeError("unsupported FD-NN shape")
        self.n_fft, self.users = n_fft, users
        self.max_sym = int(max_sym)
        self.device = torch.device(device)
        nb = L.fdnn_workspace_size(self.desc, self.max_sym)
        self.workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)

    def _n(self, s):
        n = s.shape[0]
        _check_c(s, (n, self.users, self.n_fft, 2), "s")
        if n > self.max_sym:
            raise ValueError("more OFDM symbols than the workspace was sized for")
        return n

    def forward(self, s, w):
        n = self._n(s)
        out = torch.empty_like(s)
        L.fdnn_forward(self.desc, n, s, w, out, self.workspace)
        return out

    def backward(self, s, w, g_out):
        n = self._n(s)
        dw = torch.empty(self.P, dtype=torch.float32, device=self.device)
        L.fdnn_backward(self.desc, n, s, w, g_out, dw, self.workspace)
        return dw


class FdNnFn(torch.autograd.Function):
    """out = FD-NN(s; w) as a function of the packed weights w (s is data)."""

    @staticmethod
    def forward(ctx, w, s, net: FdNn):
        out = net.forward(s, w.detach())
        ctx.save_for_backward(w, s)
        ctx.net = net
        return out

    @staticmethod
    def backward(ctx, grad_out):
        w, s = ctx.saved_tensors
        return ctx.net.backward(s, w.detach(), grad_out.contiguous()), None, None


class Downlink:
    def __init__(self, n_fft=4096, n_data=384, users=8, antennas=32, taps=10, qam=256, pa=(7, 3, 1),
                 dpd=None, device="cuda"):
        self.desc = L.link_desc(n_fft, n_data, users, antennas, taps, qam, L.GmpDesc(*pa),
                                L.GmpDesc(*dpd) if dpd else None)
        self.n_fft, self.n_data, self.users, self.antennas, self.taps = n_fft, n_data, users, antennas, taps
        self.device = torch.device(device)

    def zf(self, h_est, p_total, all_bins=False):
        """-> (pt [n_ch][N][B][U][2], alpha [n_ch]) from the estimated taps [n_ch][T][U][B][2];
        pt is written on the data subcarriers only unless all_bins (guard entries are zero
        then, as allocated here)."""
        n_ch = h_est.shape[0]
        _check_c(h_est, (n_ch, self.taps, self.users, self.antennas, 2), "h_est")
        alloc = torch.empty if all_bins else torch.zeros
        pt = alloc(n_ch, self.n_fft, self.antennas, self.users, 2, dtype=torch.float32, device=self.device)
        alpha = torch.empty(n_ch, dtype=torch.float32, device=self.device)
        ws = torch.empty(max(L.zf_workspace_size(self.desc, n_ch), 256), dtype=torch.uint8, device=self.device)
        L.zf_precoder(self.desc, n_ch, h_est, p_total, all_bins, pt, alpha, ws)
        return pt, alpha

    def _check_channels(self, pt, alpha, n_sym, sym_per_ch, h=None):
        n_ch = -(-n_sym // sym_per_ch)
        if pt is not None:
            _check_c(pt, (pt.shape[0], self.n_fft, self.antennas, self.users, 2), "pt")
            if pt.shape[0] < n_ch:
                raise ValueError(f"pt holds {pt.shape[0]} channel realisations, {n_ch} needed")
        if h is not None:
            _check_c(h, (h.shape[0], self.taps, self.users, self.antennas, 2), "h")
            if h.shape[0] < n_ch:
                raise ValueError(f"h holds {h.shape[0]} channel realisations, {n_ch} needed")
        if alpha.dtype != torch.float32 or alpha.numel() < n_ch:
            raise ValueError(f"alpha: float32 with at least {n_ch} entries expected")

    def precode(self, s, pt, alpha, sym_per_ch=1, all_bins=False):
        """UE symbols on the subcarriers [n_sym][U][N][2] -> antenna subcarriers [n_sym][B][N][2]."""
        n = s.shape[0]
        _check_c(s, (n, self.users, self.n_fft, 2), "s")
        self._check_channels(pt, alpha, n, sym_per_ch)
        x = torch.empty(n, self.antennas, self.n_fft, 2, dtype=torch.float32, device=self.device)
        L.ofdm_precode(self.desc, n, sym_per_ch, pt, alpha, s, all_bins, x)
        return x

    def _check_coef(self, coef, orders, name):
        K, M, L_ = orders
        J = K * (M + 1) + 2 * (K - 1) * (M + 1) * L_
        _check_c(coef, (self.antennas, J, 2), name)

    def link(self, x, pa_coef, g, h, alpha, tx, noise=None, dpd_coef=None, sym_per_ch=1, want_r=False):
        """-> (symbol errors per UE int64 [U], equalised symbols [n_sym][U][n_data][2] or None)."""
        n = x.shape[0]
        _check_c(x, (n, self.antennas, self.n_fft, 2), "x")
        self._check_coef(pa_coef, (self.desc.pa.K, self.desc.pa.M, self.desc.pa.L), "pa_coef")
        if self.desc.dpd.K:
            if dpd_coef is None:
                raise ValueError("this link has a DPD: dpd_coef is required")
            self._check_coef(dpd_coef, (self.desc.dpd.K, self.desc.dpd.M, self.desc.dpd.L), "dpd_coef")
        if noise is not None:
            _check_c(noise, (n, self.users, self.n_fft, 2), "noise")
        self._check_channels(None, alpha, n, sym_per_ch, h)
        if tx.dtype != torch.int32 or tuple(tx.shape) != (n, self.users, self.n_data) or not tx.is_contiguous():
            raise ValueError("tx: expected contiguous int32 [n_sym][U][n_data]")
        errors = torch.empty(self.users, dtype=torch.int64, device=self.device)
        r = (torch.empty(n, self.users, self.n_data, 2, dtype=torch.float32, device=self.device)
             if want_r else None)
        ws = torch.empty(max(L.link_workspace_size(self.desc, n, sym_per_ch), 256), dtype=torch.uint8,
                         device=self.device)
        L.ofdm_link(self.desc, n, sym_per_ch, x, dpd_coef, pa_coef, g, h, alpha, noise, tx, r, errors, ws)
        return errors, r

    def link_backward(self, x, pa_coef, g, h, alpha, g_r, sym_per_ch=1):
        """Gradient with respect to the precoded subcarriers x of a real loss on the
        equalised symbols, given its gradient g_r [n_sym][U][n_data][2]."""
        n = x.shape[0]
        _check_c(x, (n, self.antennas, self.n_fft, 2), "x")
        _check_c(g_r, (n, self.users, self.n_data, 2), "g_r")
        self._check_coef(pa_coef, (self.desc.pa.K, self.desc.pa.M, self.desc.pa.L), "pa_coef")
        self._check_channels(None, alpha, n, sym_per_ch, h)
        g_x = torch.empty_like(x)
        ws = torch.empty(max(L.link_workspace_size(self.desc, n, sym_per_ch), 256), dtype=torch.uint8,
                         device=self.device)
        L.ofdm_link_backward(self.desc, n, sym_per_ch, x, pa_coef, g, h, alpha, g_r, g_x, ws)
        return g_x

    def precode_backward(self, g_x, pt, alpha, sym_per_ch=1, all_bins=False):
        """Adjoint of precode: [n_sym][B][N][2] -> [n_sym][U][N][2]."""
        n = g_x.shape[0]
        _check_c(g_x, (n, self.antennas, self.n_fft, 2), "g_x")
        self._check_channels(pt, alpha, n, sym_per_ch)
        g_s = torch.empty(n, self.users, self.n_fft, 2, dtype=torch.float32, device=self.device)
        L.ofdm_precode_backward(self.desc, n, sym_per_ch, pt, alpha, g_x, all_bins, g_s)
        return g_s


def symbol_mse(z, t):
    """The library's symbol MSE (dpd_symbol_mse) of complex values z against targets t
    (contiguous float32 [..][2] of one shape): (L = sum |z - t|^2 / n as a device scalar,
    dL/dz = 2 (z - t) / n)."""
    if z.shape != t.shape or z.shape[-1] != 2 or not (z.is_contiguous() and t.is_contiguous()):
        raise ValueError("z and t must be contiguous [..][2] tensors of one shape")
    n = z.numel() // 2
    out = torch.empty(2, dtype=torch.float32, device=z.device)
    grad = torch.empty_like(z)
    ws = torch.empty(max(L.dpd_symbol_mse_workspace_size(n), 256), dtype=torch.uint8, device=z.device)
    L.dpd_symbol_mse(n, z, t, out, grad, ws)
    return out[0], grad


def receiver_loss_grad(dl: Downlink, net: FdNn, s, tx, w, pt, alpha, pa_coef, g, h, sym_per_ch=1):
    """The supervised criterion of Sec. V-A-2 for the FD-NN, on the device: the UE symbols s
    through the FD-NN, guard-band ZF precoding (every subcarrier), the link (PAs, channel)
    to the equalised data symbols r; L = sum |r - s_data|^2 / (n_sym U N_d).
    Returns (L as a device scalar, dL/dw, symbol errors per UE)."""
    n = s.shape[0] * dl.users * dl.n_data
    v = net.forward(s, w)
    x = dl.precode(v, pt, alpha, sym_per_ch=sym_per_ch, all_bins=True)
    errors, r = dl.link(x, pa_coef, g, h, alpha, tx, sym_per_ch=sym_per_ch, want_r=True)
    bins = torch.as_tensor(_data_bins(dl.n_fft, dl.n_data), device=s.device)
    loss, g_r = symbol_mse(r, s.index_select(2, bins).contiguous())
    g_x = dl.link_backward(x, pa_coef, g, h, alpha, g_r, sym_per_ch=sym_per_ch)
    g_v = dl.precode_backward(g_x, pt, alpha, sym_per_ch=sym_per_ch, all_bins=True)
    return loss, net.backward(s, w, g_v), errors


def receiver_loss_grad_fdcnn(dl: Downlink, net, s, tx, w, pt, alpha, pa_coef, g, h, sym_per_ch=1):
    """The same criterion for the FD-CNN (Sec. IV-A, trained like the FD-NN, Sec. V-A-2):
    each UE's N_d data symbols (items = n_sym x U symbol vectors) through the FD-CNN, back
    on the data subcarriers, data-only ZF precoding, the link; L as above.  `net` is an
    FdCnn for n_d = dl.n_data.  Returns (L, dL/dw, symbol errors per UE)."""
    n_sym = s.shape[0]
    n = n_sym * dl.users * dl.n_data
    bins = torch.as_tensor(_data_bins(dl.n_fft, dl.n_data), device=s.device)
    s_data = s.index_select(2, bins).contiguous()                       # [n_sym][U][N_d][2]
    items = s_data.view(n_sym * dl.users, dl.n_data, 2)
    v = net.forward(items, w).view(n_sym, dl.users, dl.n_data, 2)
    v_full = torch.zeros_like(s)
    v_full.index_copy_(2, bins, v)
    x = dl.precode(v_full, pt, alpha, sym_per_ch=sym_per_ch, all_bins=False)
    errors, r = dl.link(x, pa_coef, g, h, alpha, tx, sym_per_ch=sym_per_ch, want_r=True)
    loss, g_r = symbol_mse(r, s_data)
    g_x = dl.link_backward(x, pa_coef, g, h, alpha, g_r, sym_per_ch=sym_per_ch)
    g_v = dl.precode_backward(g_x, pt, alpha, sym_per_ch=sym_per_ch, all_bins=False)
    g_items = g_v.index_select(2, bins).contiguous().view(n_sym * dl.users, dl.n_data, 2)
    return loss, net.backward(items, w, g_items), errors


def train_receiver(dl: Downlink, net: FdNn, s, tx, w, pt, alpha, pa_coef, g, h, steps, lr=1e-3,
                   sym_per_ch=1, state=None):
    """`steps` device Adam updates of w in place on the receiver-side loss (the paper trains
    the FD-NN and the FD-CNN this way, Adam with learning rate 0.001); `net` is an FdNn
    (precoding on every subcarrier) or an FdCnn (data subcarriers).  Returns the loss before each step
    (device [steps]), the symbol errors before each step (device [steps][U]) and the
    optimiser state (m, v, t)."""
    m, v, t = (torch.zeros_like(w), torch.zeros_like(w), 0) if state is None else state
    losses = torch.empty(steps, dtype=torch.float32, device=w.device)
    errs = torch.empty(steps, dl.users, dtype=torch.int64, device=w.device)
    crit = receiver_loss_grad if isinstance(net, FdNn) else receiver_loss_grad_fdcnn
    for i in range(steps):
        loss, dw, e = crit(dl, net, s, tx, w, pt, alpha, pa_coef, g, h, sym_per_ch)
        losses[i] = loss
        errs[i] = e
        t += 1
        L.dpd_adam_step(dw, w, m, v, t, lr=lr)
    return losses, errs, (m, v, t)


def _data_bins(n_fft, n_d):
    """Subcarriers of the data symbols in symbol order: 1..n_d/2, then n_fft - n_d/2.."""
    h = n_d // 2
    return list(range(1, h + 1)) + list(range(n_fft - h, n_fft))
