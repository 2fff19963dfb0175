"""FWI gradient with respect to squared slowness m = 1/v^2 (adjoint-state method).

The forward model is the leapfrog step of the library (Dirichlet halos, optional
sponge), a Ricker source and receivers; the misfit is any function of the synthetic
traces.  ``FWIGrad.apply(m, problem)`` returns the traces and, on ``backward``, the
gradient of the loss with respect to m, computed by

* a forward sweep that keeps ``(u^{n-1}, u^n)`` every ``checkpoint_every`` steps
  (one native step loop, fd_forward_run, per checkpoint interval),
* a reverse sweep over the segments, last first: each segment's wavefields are
  recomputed from its checkpoint into a segment buffer, then for n descending the
  adjoint step forms the adjoint field at n from those at n+1 and n+2 with the
  gradient accumulation fused in, and the trace residual of step n-1 is added at
  the receivers,
* the final scaling of the accumulated gradient to grad_m.

The adjoint runs by default in the scaled variable b = vdt2 D lambda
(``fd_adjoint_step_scaled``, ``fd_scatter_add_scaled``, ``fd_grad_finalize_scaled``):
there it is the forward update run backward in time, on the forward kernel, and
g_b = sum b^{n+1} (L u^n + f^n) gives grad_m = -g_b vdt2 / dt^2.  ``scaled=False``
runs it in lambda (``fd_adjoint_step``: lambda^n = 2 D lambda^{n+1} +
L(vdt2 D lambda^{n+1}) - E D lambda^{n+2}, g += D lambda^{n+1} (L u^n + f^n),
``fd_scatter_add``, ``fd_grad_finalize``: grad_m = -g vdt2^2 / dt^2).

dt and the sponge are fixed when the problem is built (they do not depend on m).
All device work runs in libfd's kernels; torch allocates buffers and copies
checkpoints.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api

# grids up to this many points run short, latency-bound launches: there the receiver
# residual is added in the adjoint update's own launch (fd_adjoint_step_scaled_res),
# as it is on grids the 16-byte-lane kernel steps (it loads the residual row before it
# marches); the marching kernel of one float per lane in between would wait for its
# map lookup, and a separate launch costs less there
SMALL_GRID_POINTS = 1 << 20


class FWIProblem:
    """One shot of an FWI gradient: geometry, time axis, source, receivers."""

    def __init__(self, shape, dt: float, src, rec: np.ndarray, nt: int, d=(10.0, 10.0, 10.0),
                 sponge_width: int = 16, sponge_vmax: float | None = None,
                 f0: float = api.RICKER_F0, t0: float | None = None,
                 checkpoint_every: int = 32, device="cuda"):
        nx, ny, nz = shape
        self.grid = g = api.Grid(nx, ny, nz, d)
        self.dt = float(dt)
        self.nt = int(nt)
        self.src = tuple(int(x) for x in src)
        self.device = device
        # checkpoint_every = 0 keeps every state u^0 .. u^{nt-1} (nt volumes: 89 GB
        # at 256^3 and 1000 steps fits one MI355X's 288 GB) and skips the recompute
        self.C = int(checkpoint_every)
        if self.C < 0:
            raise ValueError("checkpoint_every must be >= 0 (0: keep every state)")
        if sponge_width > 0:
            if sponge_vmax is None:
                raise ValueError("a sponge needs the (fixed) vmax it is designed for")
            self.sponge = api.Sponge(g, sponge_width, sponge_vmax, self.dt, device=device)
        else:
            self.sponge = None
        self.w = api.ricker(self.nt, self.dt, f0, t0)
        self.rec_off = torch.from_numpy(g.offsets(rec)).to(device)
        self.rec_plane = api.receiver_plane(g, rec, device)  # sampled in the stencil launch
        self.nrec = self.rec_off.numel()
        self.src_off = torch.from_numpy(g.offsets(np.array([self.src], np.int32))).to(device)
        self.m = g.zeros(device)
        self.vdt2 = g.zeros(device)
        self.ckpt: list[tuple[torch.Tensor, torch.Tensor]] = []
        self.states: list[torch.Tensor] = []

    # ------------------------------------------------------------ forward
    def set_model(self, m_interior: torch.Tensor):
        g = self.grid
        g.interior(self.m).copy_(m_interior.detach())
        # only m's interior is read: vdt2's face halos take its periodic image
        api.prepare_vdt2_m(g, self.m, self.vdt2, self.dt)

    def forward(self, m_interior: torch.Tensor, checkpoints: bool = True) -> torch.Tensor:
        """Traces (nt, nrec) of the model m; keeps checkpoints for ``backward``."""
        g = self.grid
        self.set_model(m_interior)
        up, u, un = g.zeros(self.device), g.zeros(self.device), g.zeros(self.device)
        traces = torch.zeros((self.nt, self.nrec), dtype=torch.float32, device=self.device)
        self.ckpt = []
        if checkpoints and self.C == 0:
            return self._forward_store_all(traces)
        self.states = []
        step = self.C if self.C > 0 else self.nt
        for s in range(0, self.nt, step):  # one native loop per checkpoint interval
            e = min(s + step, self.nt)
            if checkpoints:
                self.ckpt.append((up.clone(), u.clone()))
            up, u, un = api.forward_run(g, up, u, un, self.vdt2, self.sponge, e - s,
                                        src=self.src, wavelet=self.w[s:e],
                                        rec_off=self.rec_off, traces=traces[s:e],
                                        rec_plane=self.rec_plane)
        return traces

    def _forward_store_all(self, traces: torch.Tensor) -> torch.Tensor:
        """Forward sweep writing u^{n+1} of step n into its own buffer: states[n] is
        u^n for n < nt (states[0] = u^0 = 0); u^{nt} lands in a spare buffer."""
        g = self.grid
        if len(self.states) != self.nt + 2:
            self.states = []
            torch.cuda.empty_cache()
            self.states = [g.zeros(self.device) for _ in range(self.nt + 2)]
        else:
            self.states[0].zero_()
            self.states[-1].zero_()
        zero = self.states[-1]  # u^{-1}
        for n in range(self.nt):
            up = zero if n == 0 else self.states[n - 1]
            api.step_fused(g, up, self.states[n], self.states[n + 1], self.vdt2, self.sponge,
                           (self.src, float(self.w[n])))
            api.record_receivers(g, self.states[n + 1], self.rec_off, traces[n])
        return traces

    # ------------------------------------------------------------ adjoint
    def backward(self, res: torch.Tensor, want_grad_w: bool = False, scaled: bool = True,
                 want_lambda_src: bool = False):
        """grad_m (interior, float32) for trace residual ``res`` (nt, nrec) = dLoss/dtraces.

        ``scaled`` (default) runs the adjoint in b = vdt2 D lambda, where it is the
        forward update run backward in time (fd_adjoint_step_scaled); with
        ``want_grad_w`` it also returns dLoss/dw[n] = b^{n+1} at the source.
        ``scaled=False`` runs it in lambda itself (fd_adjoint_step); with
        ``want_lambda_src`` it also returns lambda^{n+1} at the source."""
        if scaled and want_lambda_src or not scaled and want_grad_w:
            raise ValueError("want_grad_w goes with scaled=True, want_lambda_src with False")
        g = self.grid
        nt, C = self.nt, self.C
        if not self.ckpt and not (C == 0 and self.states):
            raise RuntimeError("backward needs a forward run with checkpoints")
        res = res.to(device=self.device, dtype=torch.float32).contiguous()
        if res.shape != (nt, self.nrec):
            raise ValueError(f"residual must be ({nt}, {self.nrec})")
        if scaled:
            return self._backward_scaled(res, want_grad_w)
        A = g.zeros(self.device)  # lambda^{n+2}
        B = g.zeros(self.device)  # lambda^{n+1}
        api.scatter_add(g, B, self.rec_off, res[nt - 1])
        gq = g.zeros(self.device)
        seg = self._segment_buffers()
        lam_src = torch.zeros(nt, dtype=torch.float32, device=self.device) if want_lambda_src else None
        for j in range(self._segments() - 1, -1, -1):
            s, e, seg = self._recompute(j, seg)
            for n in range(e - 1, s - 1, -1):
                if lam_src is not None:
                    api.record_receivers(g, B, self.src_off, lam_src[n:n + 1])
                api.adjoint_step(g, A, B, A, self.vdt2, self.sponge, u_n=seg[n - s], g_vdt2=gq,
                                 src=(self.src, float(self.w[n])))
                if n >= 1:
                    api.scatter_add(g, A, self.rec_off, res[n - 1])
                A, B = B, A
        gm = g.zeros(self.device)
        api.grad_finalize(g, gq, self.vdt2, self.dt, gm)
        out = g.interior(gm).clone()
        if want_lambda_src:
            return out, lam_src
        return out

    def _segments(self) -> int:
        return 1 if self.C == 0 else len(self.ckpt)

    def _segment_buffers(self) -> list[torch.Tensor]:
        if self.C == 0:
            return []
        return [self.grid.zeros(self.device) for _ in range(min(self.C, self.nt))]

    def _recompute(self, j: int, seg: list[torch.Tensor]):
        """(s, e, buffers) with buffers[i] = u^{s+i} for segment j: the stored states,
        or u^s .. u^{e-1} recomputed into ``seg`` from the segment's checkpoint."""
        if self.C == 0:
            return 0, self.nt, self.states
        g, C = self.grid, self.C
        s = j * C
        e = min(s + C, self.nt)
        prev, cur = self.ckpt[j]
        seg[0].copy_(cur)
        before = prev
        for n in range(s, e - 1):
            i = n - s
            api.step_fused(g, before, seg[i], seg[i + 1], self.vdt2, self.sponge,
                           (self.src, float(self.w[n])))
            before = seg[i]
        return s, e, seg

    @property
    def _inject_in_step(self) -> bool:
        g = self.grid
        if self.rec_plane is None:
            return False
        return (g.nx * g.ny * g.nz <= SMALL_GRID_POINTS
                or api.step_kernel(g)["kernel"] in ("wide_128x32", "wide_64x64"))

    def _backward_scaled(self, res: torch.Tensor, want_grad_w: bool):
        g, nt = self.grid, self.nt
        A = g.zeros(self.device)  # b^{n+2}
        B = g.zeros(self.device)  # b^{n+1}
        api.scatter_add_scaled(g, B, self.rec_off, res[nt - 1], self.vdt2, self.sponge)
        gb = g.zeros(self.device)
        seg = self._segment_buffers()
        grad_w = torch.zeros(nt, dtype=torch.float32, device=self.device) if want_grad_w else None
        in_step = self._inject_in_step
        for j in range(self._segments() - 1, -1, -1):
            s, e, seg = self._recompute(j, seg)
            for n in range(e - 1, s - 1, -1):
                if grad_w is not None:
                    api.record_receivers(g, B, self.src_off, grad_w[n:n + 1])
                # the residual of step n-1 enters at the receivers: in the update's own
                # launch when they share one plane (see SMALL_GRID_POINTS), else by a
                # separate launch
                inj = (self.rec_plane, res[n - 1]) if n >= 1 and in_step else None
                api.adjoint_step_scaled(g, A, B, A, self.vdt2, self.sponge, u_n=seg[n - s],
                                        g_b=gb, src=(self.src, float(self.w[n])), res=inj)
                if n >= 1 and inj is None:
                    api.scatter_add_scaled(g, A, self.rec_off, res[n - 1], self.vdt2,
                                           self.sponge)
                A, B = B, A
        api.grad_finalize_scaled(g, gb, self.vdt2, self.dt, gb)
        out = g.interior(gb).clone()
        if want_grad_w:
            return out, grad_w
        return out


class FWIGrad(torch.autograd.Function):
    """traces = FWIGrad.apply(m, problem); m is the (nz, ny, nx) interior of the
    squared slowness on the device.  backward gives dLoss/dm."""

    @staticmethod
    def forward(ctx, m: torch.Tensor, problem: FWIProblem):
        ctx.problem = problem
        return problem.forward(m)

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        return ctx.problem.backward(grad_traces), None


def misfit_gradient(problem: FWIProblem, m: torch.Tensor, obs: torch.Tensor):
    """J = 1/2 sum (traces - obs)^2 (accumulated in float64) and dJ/dm."""
    m = m.detach().clone().requires_grad_(True)
    tr = FWIGrad.apply(m, problem)
    r = tr - obs
    J = 0.5 * float((r.double() ** 2).sum().item())
    tr.backward(r)
    return J, m.grad
