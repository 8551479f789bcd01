"""Differentiable currents: a torch.autograd.Function whose forward runs the
path (wt_h_solve, wt_current) and whose backward is the library's hand-written
adjoint (wt_h_gradient).

The parameters are, per column, its quarter-column resistivities and its
radius, packed as a CPU float64 tensor theta[n_cols][5]: resistivity[p] (ohm
m) in slots p < n_resistivity, the radius (m) in slot 4; unused slots are
ignored and get a zero gradient; and the pitch (a CPU float64 scalar tensor,
m): the in-plane cell size L_x, with L_y, the column axes and the carriers'
in-plane coordinates scaled by the same factor.  The backward reads only the solve's
workspace (collocation matrix, charges q(w), field table): H is released as
soon as the currents are computed and is never recomputed, so the forward's
FFT stages need no storage at all in the backward.

Argument marshalling only; every step runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import wt


class _Plan:
    """Owns a plan handle and the device workspace of one forward solve."""

    def __init__(self, handle, layout, ws):
        self.handle, self.layout, self.ws = handle, layout, ws

    def __del__(self):
        try:
            wt.wt_h_plan_destroy(self.handle)
        except Exception:
            pass


class ColumnModel:
    """A pixel cell, its columns, the frequency/time grid and the carriers.

    carriers: dict with pos [n_c][n_time+1][3], charge [n_c], track [n_c]
    (numpy or torch) and n_tracks; they are copied to the device once.
    """

    def __init__(self, cell, columns, spectrum, carriers, precision=wt.WT_F32, ir_max_iter=2, ir_tol=1e-12):
        self.cell, self.columns, self.spectrum = cell, [dict(c) for c in columns], spectrum
        self.precision, self.ir_max_iter, self.ir_tol = precision, ir_max_iter, ir_tol
        self.dtype = torch.float64 if precision == wt.WT_F64 else torch.float32
        dev = torch.device("cuda", torch.cuda.current_device())
        self.pos = torch.as_tensor(np.asarray(carriers["pos"])).to(dev, self.dtype).contiguous()
        self.charge = torch.as_tensor(np.asarray(carriers["charge"])).to(dev, self.dtype).contiguous()
        self.track = torch.as_tensor(np.asarray(carriers["track"], dtype=np.int32)).to(dev).contiguous()
        self.n_tracks = int(carriers["n_tracks"])
        self.ctx = wt.wt_context_create(dev.index, torch.cuda.current_stream().cuda_stream)

    def __del__(self):
        try:
            wt.wt_context_destroy(self.ctx)
        except Exception:
            pass

    def theta0(self):
        """The model's own parameters as theta[n_cols][5] (CPU float64)."""
        th = torch.zeros((len(self.columns), 5), dtype=torch.float64)
        for w, c in enumerate(self.columns):
            for p, r in enumerate(c["resistivity"]):
                th[w, p] = r
            th[w, 4] = c["radius"]
        return th

    def columns_at(self, theta):
        th = theta.detach().cpu().numpy()
        out = []
        for w, c in enumerate(self.columns):
            n = len(c["resistivity"])
            out.append(dict(c, resistivity=[float(th[w, p]) for p in range(n)], radius=float(th[w, 4])))
        return out

    def pitch0(self):
        """The model's own pitch (L_x) as a CPU float64 scalar tensor."""
        return torch.tensor(float(self.cell["L"][0]), dtype=torch.float64)

    def geometry_at(self, theta, pitch=None):
        """(cell, columns, positions) at theta and pitch (positions on the device)."""
        cols = self.columns_at(theta)
        if pitch is None:
            return self.cell, cols, self.pos
        s = float(pitch) / float(self.cell["L"][0])
        if s == 1.0:
            return self.cell, cols, self.pos
        L = self.cell["L"]
        cell = dict(self.cell, L=(L[0] * s, L[1] * s, L[2]))
        cols = [dict(c, x=c["x"] * s, y=c["y"] * s) for c in cols]
        pos = self.pos.clone()
        pos[..., :2] *= s
        return cell, cols, pos

    def solve(self, theta, pitch=None):
        """Plan, solve and currents at theta (and pitch) -> (_Plan, currents [n_tracks][n_time])."""
        cell, cols, pos = self.geometry_at(theta, pitch)
        handle, lay = wt.wt_h_plan_create(cell, cols, self.spectrum, self.precision, self.ir_max_iter, self.ir_tol)
        ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device=self.pos.device)
        plan = _Plan(handle, lay, ws)
        hbuf = torch.empty(lay["h_bytes"], dtype=torch.uint8, device=self.pos.device)
        wt.wt_h_solve(self.ctx, handle, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel())
        out = torch.empty((self.n_tracks, self.spectrum["n_time"]), dtype=self.dtype, device=self.pos.device)
        cws = torch.empty(wt.wt_current_workspace(handle, pos.shape[0]), dtype=torch.uint8, device=self.pos.device)
        wt.wt_current(self.ctx, handle, hbuf.data_ptr(), pos.shape[0], self.n_tracks, pos.data_ptr(),
                      self.charge.data_ptr(), self.track.data_ptr(), out.data_ptr(), cws.data_ptr(), cws.numel())
        plan.pos = pos
        # H is consumed in stream order; dropping the last reference lets the
        # caching allocator reuse it for work enqueued after this point.
        del hbuf, cws
        return plan, out

    def gradient(self, plan, grad_current):
        """(dL/dtheta [n_cols][5], dL/dpitch []) (CPU float64) for dL/di on the device."""
        g = grad_current.to(self.dtype).contiguous()
        nbytes = wt.wt_h_gradient_workspace(plan.handle, self.n_tracks)
        gws = torch.empty(nbytes, dtype=torch.uint8, device=self.pos.device)
        n = len(self.columns)
        out = torch.empty(5 * n + 1, dtype=torch.float64, device=self.pos.device)
        pos = plan.pos
        wt.wt_h_gradient(self.ctx, plan.handle, plan.ws.data_ptr(), plan.ws.numel(), pos.shape[0],
                         self.n_tracks, pos.data_ptr(), self.charge.data_ptr(), self.track.data_ptr(),
                         g.data_ptr(), gws.data_ptr(), nbytes, out.data_ptr())
        out = out.cpu()
        return out[:5 * n].view(n, 5), out[5 * n]

    def currents(self, theta, pitch=None):
        """Differentiable currents [n_tracks][n_time] on the device."""
        if pitch is None:
            pitch = self.pitch0()
        return ColumnCurrents.apply(theta, pitch, self)


class ColumnCurrents(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, pitch, model):
        plan, out = model.solve(theta, pitch)
        ctx.plan, ctx.model = plan, model
        return out

    @staticmethod
    def backward(ctx, grad_out):
        g_theta, g_pitch = ctx.model.gradient(ctx.plan, grad_out)
        return g_theta, g_pitch, None


def signal_features(i, dt, t_center, t_sigma, t_max):
    """Per-track peak time and windowed charge of currents i [n_tracks][n_time].

    t_peak: the first index of max |i| refined by the vertex of the parabola
    through the three samples around it (the index itself is piecewise
    constant, so its derivative is that of the vertex offset);
    q_w: the rectangle-rule integral of i(t) w(t) over [0, t_max] with the
    Gaussian window w(t) = exp(-(t - t_center)^2 / (2 t_sigma^2)).
    """
    n_t = i.shape[1]
    t = torch.arange(n_t, device=i.device, dtype=i.dtype) * dt
    w = torch.exp(-(t - t_center) ** 2 / (2.0 * t_sigma ** 2)) * (t <= t_max + 0.5 * dt)
    q_w = (i * w).sum(dim=1) * dt
    n_p = torch.argmax(i.detach().abs(), dim=1).clamp(1, n_t - 2)
    s = torch.sign(i.gather(1, n_p[:, None]).detach())
    um = (s * i.gather(1, (n_p - 1)[:, None]))[:, 0]
    u0 = (s * i.gather(1, n_p[:, None]))[:, 0]
    up = (s * i.gather(1, (n_p + 1)[:, None]))[:, 0]
    d = 0.5 * (um - up) / (um - 2.0 * u0 + up)
    t_peak = (n_p.to(i.dtype) + d) * dt
    return t_peak, q_w
