"""Run the hot path on a workload through the C-ABI and return numpy results.

Used by the tests, the smoke check and the bench.  A workload is any object
with ``mesh`` (CSR arrays), ``alpha``, ``T``, ``T_bface``, ``T_sat``, ``k_l``,
``k_v`` and ``h_lv``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import vofpc as V


class PathRun:
    """Device-resident inputs and buffers of one workload, ready to step."""

    def __init__(self, wl, device: int = 0, opts: V.ReconOpts | None = None, ctx: V.Context | None = None,
                 hint_lo=None, hint_hi=None, mlp: "V.Mlp | None" = None, delta_scale: float = 0.0,
                 parts: list | None = None):
        """`parts`: the meshes whose disjoint union is wl.mesh; each is uploaded
        on its own and the library concatenates them on the device."""
        self.dev = torch.device("cuda", device)
        # a stream of its own (default priority): graph capture needs a
        # non-null stream
        self.ctx = ctx or V.Context(device, stream=torch.cuda.Stream(self.dev))
        if parts:
            ups = [V.Mesh(self.ctx, m) for m in parts]
            self.mesh = V.Mesh.concat(self.ctx, ups)
            for u in ups:
                u.close()
        else:
            self.mesh = V.Mesh(self.ctx, wl.mesh)
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.alpha = torch.as_tensor(np.ascontiguousarray(wl.alpha), **f64)
        self.T = torch.as_tensor(np.ascontiguousarray(wl.T), **f64)
        self.Tb = torch.as_tensor(np.ascontiguousarray(wl.T_bface), **f64)
        self.buf = V.StepBuffers(self.ctx, self.mesh, self.alpha, self.T, self.Tb, wl.T_sat, wl.k_l, wl.k_v,
                                 wl.h_lv, opts=opts, hint_lo=hint_lo, hint_hi=hint_hi, mlp=mlp,
                                 delta_scale=delta_scale)
        torch.cuda.synchronize(self.dev)   # inputs were written on torch's stream
        self.graph = None

    def step(self) -> None:
        V.step(self.ctx, self.mesh, self.buf)

    def capture(self) -> V.Graph:
        if self.graph is None:
            self.graph = V.Graph(self.ctx, self.mesh, self.buf)
        return self.graph

    def results(self) -> dict:
        """Synchronise and copy the step outputs to host numpy arrays."""
        torch.cuda.synchronize(self.dev)
        b = self.buf
        nm, nb = (int(x) for x in b.counts.cpu())
        itf = b.itf
        out = dict(
            n_mixed=nm, n_band=nb,
            mixed_idx=b.mixed_idx[:nm].cpu().numpy(), band_idx=b.band_idx[:nb].cpu().numpy(),
            s=itf.s[:nm].cpu().numpy(), n=itf.n[:, :nm].cpu().numpy(), A=itf.A[:nm].cpu().numpy(),
            d=itf.d[:nm].cpu().numpy(), alpha_got=itf.alpha_got[:nm].cpu().numpy(),
            status=itf.status[:nm].cpu().numpy(), iters=itf.iters[:nm].cpu().numpy(),
            gradT=b.gradT.cpu().numpy(), grad_status=b.grad_status.cpu().numpy(),
            mdot=b.mdot[:nm].cpu().numpy(), Qdot=b.Qdot[:nm].cpu().numpy(),
        )
        return out

    def close(self) -> None:
        if self.graph is not None:
            self.graph.close()
        self.mesh.close()
