"""Differentiable multi-step MFM evolution: torch.autograd.Function over the
library's fixed-dt kick-drift-kick steps, with the hand-written adjoint.

Forward runs the initial pass and k steps on the GPU and keeps one checkpoint
of the state per step (positions, velocities, energies, kernel lengths and the
pass outputs dp, dE).  With `tape` (the default) each step also records its
tape (mfm_step_taped: the step's predicted state, pass outputs, permutation and
flux lists, about 1.4 kB per particle with 256 list slots), and the backward
reads it (mfm_step_adjoint_taped); without, each mfm_step_adjoint recomputes
its step from the checkpoint.  Backward walks the steps from last to first;
the initial pass is reversed last with mfm_hydro_pass_adjoint.
Only v and u of the initial state are differentiable inputs; positions and
masses are fixed data.
"""
from __future__ import annotations

import torch

from . import mfm

_CK = ("x", "y", "z", "m", "vx", "vy", "vz", "u", "H", "dp", "dE", "id")


def _copy_state(dst: mfm.State, src: mfm.State):
    # one multi-tensor copy per dtype instead of a copy per array
    f64 = [k for k in _CK if k != "id"]
    torch._foreach_copy_([getattr(dst, k) for k in f64], [getattr(src, k) for k in f64])
    dst.id.copy_(src.id)


class Evolution:
    """Fixed data of one differentiable run: positions, masses, parameters."""

    def __init__(self, w, steps: int, dt: float, cfg: mfm.Config | None = None, tape: bool = True):
        self.w = w
        self.steps = int(steps)
        self.dt = float(dt)
        self.tape = bool(tape)
        self.cfg = cfg or mfm.config_of(w)
        self.ctx = mfm.Context(self.cfg, w.n)
        self.n = w.n
        # the fixed data, resident on the device once
        self.dev = {k: torch.as_tensor(v, dtype=torch.float64).cuda() for k, v in w.arrays().items()}

    def _state(self):
        # every checkpoint array is copied in before it is read
        return mfm.State(self.n, zero=False)

    def run(self, v0: torch.Tensor, u0: torch.Tensor, keep: bool):
        """Forward; v0 (3, n) and u0 (n) in the input order.  Returns the final
        state (library order) and, if keep, the checkpoints (with each step's
        tape as `ck.tape` when taping)."""
        st = mfm.State(self.n, zero=False)
        torch._foreach_copy_([st.x, st.y, st.z, st.m, st.vx, st.vy, st.vz, st.u],
                             [self.dev["x"], self.dev["y"], self.dev["z"], self.dev["m"], v0[0], v0[1], v0[2], u0])
        st.H.zero_()                        # cold kernel-length start
        self.ctx.build_neighbours(st)
        self.ctx.hydro_pass(st)
        cks = []
        nb = self.ctx.tape_bytes() if (keep and self.tape) else 0
        for _ in range(self.steps):
            if keep:
                ck = self._state()
                _copy_state(ck, st)
                cks.append(ck)
                if self.tape:
                    ck.tape = torch.empty(nb, dtype=torch.uint8, device="cuda")
                    self.ctx.step_taped(st, self.dt, ck.tape)
                    continue
            self.ctx.step(st, self.dt)
        return st, cks


class MFMSteps(torch.autograd.Function):
    """(v0 (3, n), u0 (n)) -> (v_k (3, n), u_k (n)) after k fixed-dt steps, both
    in the input order, differentiable through the hand-written adjoint."""

    @staticmethod
    def forward(ctx, v0, u0, evo: Evolution):
        st, cks = evo.run(v0.detach(), u0.detach(), keep=True)
        ids = st.id
        vk = torch.empty_like(v0)
        uk = torch.empty_like(u0)
        vk[:, ids] = torch.stack([st.vx, st.vy, st.vz])
        uk[ids] = st.u
        ctx.evo = evo
        ctx.cks = cks
        ctx.final_ids = ids.clone()
        return vk, uk

    @staticmethod
    def backward(ctx, gv, gu):
        evo = ctx.evo
        n = evo.n
        f = dict(dtype=torch.float64, device="cuda")
        ids = ctx.final_ids
        gv = torch.zeros(3, n, **f) if gv is None else gv.contiguous()
        gu = torch.zeros(n, **f) if gu is None else gu.contiguous()
        # adjoints in the library order of the final state
        ax = torch.zeros(3, n, **f)
        av = gv[:, ids].contiguous()
        au = gu[ids].contiguous()
        ap = torch.zeros(3, n, **f)
        ae = torch.zeros(n, **f)
        work = None
        for ck in reversed(ctx.cks):
            tape = getattr(ck, "tape", None)
            if tape is not None:
                evo.ctx.step_adjoint_taped(ck, tape, evo.dt, ax, av, au, ap, ae)
                ck.tape = None
                continue
            if work is None:
                work = mfm.State(n, zero=False)   # the step adjoint writes it before reading
            evo.ctx.step_adjoint(ck, work, evo.dt, ax, av, au, ap, ae)
        # the initial pass produced (dp, dE) of the first state: reverse it
        st0 = mfm.State(n, zero=False)
        first = ctx.cks[0] if ctx.cks else None
        if first is None:
            raise RuntimeError("MFMSteps needs at least one step")
        _copy_state(st0, first)
        evo.ctx.build_neighbours(st0)
        evo.ctx.hydro_pass(st0)
        fx, fv, fu = evo.ctx.pass_adjoint(st0, ap, ae)
        # st0 keeps the checkpoint order (it is already sorted), so the adjoints line up
        av = av + fv
        au = au + fu
        ids0 = st0.id
        g_v0 = torch.empty(3, n, **f)
        g_u0 = torch.empty(n, **f)
        g_v0[:, ids0] = av
        g_u0[ids0] = au
        ctx.cks = None
        return g_v0, g_u0, None
