"""TD-GMP benchmark DPD identified by indirect learning with least squares, on the device.

`GmpIla` holds the DPD and PA GMP descriptors, the batch and a workspace (allocated once
through torch).  One ILA iteration (Sec. V-A-2 with the GMP DPD of Sec. III-B, eq. (9)):
u = DPD(x) (pa_gmp_forward with the DPD coefficients), y = PA(u) (pa_gmp_forward with
the PA coefficients), NMSE of y against G x (cascade_nmse), then the post-inverse fit
gmp_ls_fit(z = y / G -> t = u) gives the next DPD coefficients.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


class GmpIla:
    def __init__(self, dpd_orders, pa_orders, offsets, per_stream_params=False, gain=1.0 + 0.0j,
                 device="cuda"):
        self.dpd = L.gmp_desc(*dpd_orders)
        self.pa_desc = L.gmp_desc(*pa_orders)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.batch = L.make_batch(self.offsets, per_stream_params)
        self.S = int(self.offsets.size - 1)
        self.n_sets = self.S if per_stream_params else 1
        self.n_total = int(self.offsets[-1])
        self.J = L.dpd_gmp_coeff_count(self.dpd)
        self.Jp = L.dpd_gmp_coeff_count(self.pa_desc)
        self.gain = complex(gain)
        self.device = torch.device(device)
        nb = max(L.gmp_ls_workspace_size(self.dpd, self.batch),
                 L.dpd_workspace_size(None, None, self.batch))
        self.workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)

    def identity(self):
        """DPD coefficients of the identity map (a_00 = 1 in every set)."""
        c = torch.zeros((self.n_sets, self.J, 2), dtype=torch.float32, device=self.device)
        c[:, 0, 0] = 1.0
        return c

    def fit(self, y, t, ridge=0.0, want_normal=False):
        """Post-distorter least squares: returns (coef [n_sets][J][2], info [n_sets], normal or None)."""
        coef = torch.empty((self.n_sets, self.J, 2), dtype=torch.float32, device=self.device)
        info = torch.empty(self.n_sets, dtype=torch.int32, device=self.device)
        normal = (torch.empty((self.n_sets, self.J, self.J + 1, 2), dtype=torch.float64, device=self.device)
                  if want_normal else None)
        L.gmp_ls_fit(self.dpd, self.batch, y, self.gain, t, ridge, coef, info, normal, self.workspace)
        return coef, info, normal

    def cascade(self, x, dpd_coef, pa_coef):
        """u = DPD(x), y = PA(u), pooled NMSE (dB) of y against G x (device scalar)."""
        u = torch.empty_like(x)
        y = torch.empty_like(x)
        L.pa_gmp_forward(self.dpd, self.batch, x, dpd_coef, u)
        L.pa_gmp_forward(self.pa_desc, self.batch, u, pa_coef, y)
        nm = torch.empty((self.S + 1, L.DPD_NMSE_FIELDS), dtype=torch.float32, device=self.device)
        L.cascade_nmse(self.batch, y, x, self.gain, nm, self.workspace)
        return u, y, nm[-1, 2]

    def run(self, x, pa_coef, iters, ridge=0.0, dpd_coef=None):
        """`iters` ILA iterations from dpd_coef (default identity).  Returns the NMSE in dB
        before each refit and after the last (device tensor [iters + 1]), the final DPD
        coefficients and the info of the last fit."""
        c = self.identity() if dpd_coef is None else dpd_coef
        hist = torch.empty(iters + 1, dtype=torch.float32, device=self.device)
        info = None
        for i in range(iters):
            u, y, nm = self.cascade(x, c, pa_coef)
            hist[i] = nm
            c, info, _ = self.fit(y, u, ridge)
        hist[iters] = self.cascade(x, c, pa_coef)[2]
        return hist, c, info
