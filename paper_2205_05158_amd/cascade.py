"""Problem object and autograd boundary over the C ABI.

`Cascade` holds the descriptors, the batch and a device workspace (allocated once
through torch, the only allocator involved) and exposes the ABI calls on torch
device tensors.  `CascadeFn` is the torch.autograd.Function of the direct-learning
loss (Sec. V-A-2): its forward runs the hand-written reverse mode of the library
(dpd_backward) together with the loss, so the backward only scales the stored
gradient by the incoming grad.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


class Cascade:
    def __init__(self, taps, n_hidden, hidden, K, M, L_, offsets, per_stream_params=False,
                 residual=False, precision="fp32", impl="tuned", gain=1.0 + 0.0j, device="cuda"):
        self.tdnn = L.tdnn_desc(taps, n_hidden, hidden, residual, precision, impl)
        self.gmp = L.gmp_desc(K, M, L_)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.batch = L.make_batch(self.offsets, per_stream_params)
        self.S = int(self.offsets.size - 1)
        self.n_sets = self.S if per_stream_params else 1
        self.n_total = int(self.offsets[-1])
        self.P = L.dpd_tdnn_param_count(self.tdnn)
        self.J = L.dpd_gmp_coeff_count(self.gmp)
        self.gain = complex(gain)
        self.device = torch.device(device)
        nbytes = L.dpd_workspace_size(self.tdnn, self.gmp, self.batch)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    # -- shape checks on the host before handing pointers to the library
    def _chk(self, t, shape, dtype=torch.float32):
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"expected contiguous {dtype} cuda tensor of shape {shape}, got "
                             f"{tuple(t.shape)} {t.dtype} {t.device}")
        return t

    def _w_shape(self):
        return (self.n_sets, self.P) if self.n_sets > 1 else (self.P,)

    def _c_shape(self):
        return (self.n_sets, self.J, 2) if self.n_sets > 1 else (self.J, 2)

    def forward_u(self, x, w):
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape())
        u = torch.empty_like(x)
        L.dpd_forward(self.tdnn, self.batch, x, w, u, self.workspace)
        return u

    def pa(self, u, coef):
        self._chk(u, (self.n_total, 2)); self._chk(coef, self._c_shape())
        y = torch.empty_like(u)
        L.pa_gmp_forward(self.gmp, self.batch, u, coef, y)
        return y

    def nmse(self, y, x):
        """NMSE records [S + 1][DPD_NMSE_FIELDS]: (E, R, NMSE dB, non-finite count) per
        stream, then pooled."""
        self._chk(y, (self.n_total, 2)); self._chk(x, (self.n_total, 2))
        out = torch.empty((self.S + 1, L.DPD_NMSE_FIELDS), dtype=torch.float32, device=self.device)
        L.cascade_nmse(self.batch, y, x, self.gain, out, self.workspace)
        return out

    def run(self, x, w, coef, want_u=True, want_y=True, want_nmse=True, want_grad=True):
        """One pass of the whole cascade; returns dict of the requested outputs."""
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape()); self._chk(coef, self._c_shape())
        dev = self.device
        u = torch.empty_like(x) if want_u else None
        y = torch.empty_like(x) if want_y else None
        nm = (torch.empty((self.S + 1, L.DPD_NMSE_FIELDS), dtype=torch.float32, device=dev)
              if want_nmse else None)
        dw = torch.empty(self._w_shape(), dtype=torch.float32, device=dev) if want_grad else None
        loss = torch.empty(self.n_sets, dtype=torch.float32, device=dev) if want_grad else None
        L.dpd_cascade(self.tdnn, self.gmp, self.batch, x, w, coef, self.gain, u, y, nm, dw, loss,
                      self.workspace)
        return {"u": u, "y": y, "nmse": nm, "dw": dw, "loss": loss}

    def loss(self, x, w, coef):
        """Pooled loss per parameter set (device [n_sets]) computed by the library
        (forward, GMP, NMSE; no reverse mode)."""
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape()); self._chk(coef, self._c_shape())
        loss = torch.empty(self.n_sets, dtype=torch.float32, device=self.device)
        L.dpd_cascade(self.tdnn, self.gmp, self.batch, x, w, coef, self.gain, None, None, None, None,
                      loss, self.workspace)
        return loss

    def autotune(self, x, w, coef, reps=3):
        """Pick this problem's launch shapes by timing on these inputs (blocks until
        done); every later call of this process on the same problem uses them."""
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape()); self._chk(coef, self._c_shape())
        return L.dpd_autotune(self.tdnn, self.gmp, self.batch, x, w, coef, self.gain, reps,
                              self.workspace)

    def tune(self):
        """Launch shapes the cascade calls of this problem use."""
        return L.dpd_tune_get(self.tdnn, self.gmp, self.batch)

    def set_tune(self, tune):
        """Install launch shapes for this problem (dict of dpd_tune fields; None resets)."""
        L.dpd_tune_set(self.tdnn, self.gmp, self.batch, tune)

    def train(self, x, w, coef, steps, lr=1e-3, state=None, stream=None):
        """Direct learning on the device: `steps` times, the gradient of the pooled NMSE
        (dpd_backward) followed by an Adam update of w in place (dpd_adam_step).  state:
        (m, v, t) from a previous call to continue, else fresh.  Returns the loss before
        each step (device tensor [steps][n_sets]) and the state (m, v, t)."""
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape()); self._chk(coef, self._c_shape())
        dev = self.device
        if state is None:
            m, v, t = torch.zeros_like(w), torch.zeros_like(w), 0
        else:
            m, v, t = state
            self._chk(m, self._w_shape()); self._chk(v, self._w_shape())
        dw = torch.empty_like(w)
        losses = torch.empty((steps, self.n_sets), dtype=torch.float32, device=dev)
        for i in range(steps):
            L.dpd_backward(self.tdnn, self.gmp, self.batch, x, w, coef, self.gain, dw, losses[i],
                           self.workspace, stream)
            t += 1
            L.dpd_adam_step(dw, w, m, v, t, lr=lr, stream=stream)
        return losses, (m, v, t)

    def backward(self, x, w, coef):
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape()); self._chk(coef, self._c_shape())
        dw = torch.empty(self._w_shape(), dtype=torch.float32, device=self.device)
        loss = torch.empty(self.n_sets, dtype=torch.float32, device=self.device)
        L.dpd_backward(self.tdnn, self.gmp, self.batch, x, w, coef, self.gain, dw, loss, self.workspace)
        return loss, dw


class ClipCascade:
    """The cascade with the ideal linear-clipping PA (Sec. V-B-2) in place of the GMP:
    DPD -> y = u below the clipping level a_clip, a_clip u / |u| above -> NMSE, with the
    library's reverse mode (dpd_cascade_clip)."""

    def __init__(self, taps, n_hidden, hidden, offsets, a_clip, per_stream_params=False, residual=False,
                 precision="fp32", impl="tuned", gain=1.0 + 0.0j, device="cuda"):
        self.tdnn = L.tdnn_desc(taps, n_hidden, hidden, residual, precision, impl)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.batch = L.make_batch(self.offsets, per_stream_params)
        self.S = int(self.offsets.size - 1)
        self.n_sets = self.S if per_stream_params else 1
        self.n_total = int(self.offsets[-1])
        self.P = L.dpd_tdnn_param_count(self.tdnn)
        self.a_clip = float(a_clip)
        self.gain = complex(gain)
        self.device = torch.device(device)
        nbytes = L.dpd_workspace_size(self.tdnn, None, self.batch)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    _chk = Cascade._chk
    _w_shape = Cascade._w_shape

    def pa(self, u):
        self._chk(u, (self.n_total, 2))
        y = torch.empty_like(u)
        L.pa_clip_forward(self.n_total, u, self.a_clip, y)
        return y

    def run(self, x, w, want_u=True, want_y=True, want_nmse=True, want_grad=True):
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape())
        dev = self.device
        u = torch.empty_like(x) if want_u else None
        y = torch.empty_like(x) if want_y else None
        nm = (torch.empty((self.S + 1, L.DPD_NMSE_FIELDS), dtype=torch.float32, device=dev)
              if want_nmse else None)
        dw = torch.empty(self._w_shape(), dtype=torch.float32, device=dev) if want_grad else None
        loss = torch.empty(self.n_sets, dtype=torch.float32, device=dev) if want_grad else None
        L.dpd_cascade_clip(self.tdnn, self.batch, x, w, self.a_clip, self.gain, u, y, nm, dw, loss,
                           self.workspace)
        return {"u": u, "y": y, "nmse": nm, "dw": dw, "loss": loss}

    def backward(self, x, w):
        out = self.run(x, w, want_u=False, want_y=False, want_nmse=False)
        return out["loss"], out["dw"]

    def train(self, x, w, steps, lr=1e-3):
        """Direct learning through the clipping PA: gradient + Adam in place, `steps` times;
        returns the loss before each step (device [steps][n_sets])."""
        self._chk(x, (self.n_total, 2)); self._chk(w, self._w_shape())
        m, v = torch.zeros_like(w), torch.zeros_like(w)
        dw = torch.empty_like(w)
        losses = torch.empty((steps, self.n_sets), dtype=torch.float32, device=self.device)
        for i in range(steps):
            L.dpd_cascade_clip(self.tdnn, self.batch, x, w, self.a_clip, self.gain, None, None, None, dw,
                               losses[i], self.workspace)
            L.dpd_adam_step(dw, w, m, v, i + 1, lr=lr)
        return losses


class CascadeFn(torch.autograd.Function):
    """loss[p] = pooled NMSE of parameter set p; differentiable w.r.t. the packed weights."""

    @staticmethod
    def forward(ctx, w, x, coef, cascade: Cascade):
        if ctx.needs_input_grad[0]:
            loss, dw = cascade.backward(x, w.detach(), coef)
            ctx.save_for_backward(dw)
        else:
            loss = cascade.loss(x, w.detach(), coef)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        (dw,) = ctx.saved_tensors
        if dw.dim() == 1:
            g = dw * grad_loss[0]
        else:
            g = dw * grad_loss[:, None]
        return g, None, None, None
