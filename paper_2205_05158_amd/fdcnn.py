"""FD-CNN DPD (Sec. IV-A) over a batch of UE symbol vectors, on the device.

`FdCnn` holds the descriptor and a workspace sized for a maximum batch (allocated once
through torch) and exposes forward, backward (parameter gradient for a given output
gradient) and a training loop against given target symbols (MSE, Adam on the device).
The paper's supervised training with the loss at the receiver, through ZF precoding,
PAs and channel, is `downlink.train_receiver` with an FdCnn.
"""
from __future__ import annotations

import torch

from . import _lib as L


class FdCnn:
    def __init__(self, n_d=384, side=20, n_conv=2, kc=3, max_items=1, device="cuda"):
        self.desc = L.FdcnnDesc(n_d, side, n_conv, kc)
        self.P = L.fdcnn_param_count(self.desc)
        if self.P < 0:
            raise RuntimeError("unsupported FD-CNN shape")
        self.n_d = n_d
        self.max_items = int(max_items)
        self.device = torch.device(device)
        nb = L.fdcnn_workspace_size(self.desc, self.max_items)
        self.workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)

    def _items(self, s):
        if s.dim() != 3 or s.shape[1:] != (self.n_d, 2) or s.dtype != torch.float32 or not s.is_contiguous():
            raise ValueError("expected contiguous float32 [items][n_d][2]")
        if s.shape[0] > self.max_items:
            raise ValueError("batch larger than the workspace was sized for")
        return s.shape[0]

    def forward(self, s, w):
        n = self._items(s)
        out = torch.empty_like(s)
        L.fdcnn_forward(self.desc, n, s, w, out, self.workspace)
        return out

    def backward(self, s, w, g_out):
        n = self._items(s)
        dw = torch.empty(self.P, dtype=torch.float32, device=self.device)
        L.fdcnn_backward(self.desc, n, s, w, g_out, dw, self.workspace)
        return dw

    def train(self, s, w, target, steps, lr=1e-3, state=None):
        """`steps` Adam updates of w in place on L = sum |out - target|^2 / (items n_d).
        Returns the loss before each step (device [steps]) and the state (m, v, t)."""
        n = self._items(s)
        if target.shape != s.shape or not target.is_contiguous():
            raise ValueError("target must be a contiguous tensor shaped like s")
        m, v, t = (torch.zeros_like(w), torch.zeros_like(w), 0) if state is None else state
        losses = torch.empty(steps, dtype=torch.float32, device=self.device)
        nv = n * self.n_d
        mse = torch.empty((steps, 2), dtype=torch.float32, device=self.device)
        g_out = torch.empty_like(s)
        ws = torch.empty(max(L.dpd_symbol_mse_workspace_size(nv), 256), dtype=torch.uint8,
                         device=self.device)
        for i in range(steps):
            out = self.forward(s, w)
            L.dpd_symbol_mse(nv, out, target, mse[i], g_out, ws)
            dw = self.backward(s, w, g_out)
            t += 1
            L.dpd_adam_step(dw, w, m, v, t, lr=lr)
        losses.copy_(mse[:, 0])
        return losses, (m, v, t)


class FdCnnFn(torch.autograd.Function):
    """out = FD-CNN(s; w) as a torch.autograd.Function of the packed parameters w: any loss
    written in torch on `out` (for instance through a precoder and channel model) reaches
    w through the library's reverse mode (fdcnn_backward).  The symbol input s is data (no
    gradient)."""

    @staticmethod
    def forward(ctx, w, s, net: FdCnn):
        out = net.forward(s, w.detach())
        ctx.save_for_backward(w, s)
        ctx.net = net
        return out

    @staticmethod
    def backward(ctx, grad_out):
        w, s = ctx.saved_tensors
        dw = ctx.net.backward(s, w.detach(), grad_out.contiguous())
        return dw, None, None
