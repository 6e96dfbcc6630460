"""Learned flood update with the finite-volume method as judge and fallback.

A small convolutional network (five 3x3 layers, BF16 MFMA kernels in libfps)
advances the flood state (h, hu, hv) by K finite-volume steps of fixed
length at once, from (h, hu, hv, z, evacuee occupancy).  This module holds
the host side of that workflow, all device work going through libfps:

* flood_case: a flood-only scenario of the shopping-centre kind (random
  building tiling, south inflow with a triangular hydrograph, random ponds so
  that water moves from the first step, optional sandbag line as raised bed)
  with a static crowd whose per-cell counts raise the Manning coefficient
  (sec. 2.3) and whose cells are where the judge looks.  The step length is
  fixed (dt_max below the CFL step), so K steps span a fixed time.
* generate_pairs / Dataset: training pairs (state at t, scaled change over
  K steps) from ensembles of such cases stepped by the finite-volume engine.
* train: Adam on the GPU with the library's forward/backward kernels.
* evaluate: held-out pairs judged at the crowd's cells against the
  finite-volume result, beside the persistence baseline (no change).
* AssistedEnsemble: the surrogate-assisted ensemble.  Per block of K steps
  the network proposes the next state of every scenario; the finite-volume
  method re-runs the K steps on the judge region only (the neighbourhoods
  of a sample of the crowd, see fps_set_judge_region); a scenario whose
  depth differs by more than 1 cm or whose hazard class (Table 1) differs at
  any sampled person falls back to the finite-volume update for that block.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import fps
from . import inputs as I

K_STEPS = 8
JUDGE_BLOCK = 16          # cells per side of a judge-region mask block
N_IN = 6                  # used input channels: h, hu, hv, z, occupancy, inflow depth
H_SNAP = 1e-3             # a dry cell stays dry unless the update puts this much water on it


@dataclasses.dataclass
class FloodCase:
    sc: I.Scenario          # flood only (no agents bound)
    agents: dict            # x, y, role, state of the static crowd
    name: str = ""


def flood_case(seed: int, n: int = 256, dx: float = 0.25, dt_s: float = 0.01, n_evac: int | None = None,
               q_peak: float | None = None, barrier_height: float | None = None, ponds: int | None = None):
    """Random flood-only case on an n x n grid (see the module docstring).
    Unset options are drawn from the seed: evacuees U(500, 5000) per 256^2
    cells, hydrograph peak U(1, 3) m^2/s over 600 s already under way,
    1-3 ponds of U(0.2, 1.0) m."""
    rng = I.rng_of(seed)
    z, walk = I.shopping_centre_layout(n, dx, seed)
    scale = n * n / 65536.0
    if n_evac is None:
        n_evac = int(rng.uniform(500, 5000) * scale)
    if q_peak is None:
        q_peak = float(rng.uniform(1.0, 3.0))
    if ponds is None:
        ponds = int(rng.integers(1, 4))
    h = np.zeros((n, n))
    for _ in range(ponds):
        w, hh = rng.integers(n // 16, n // 4, size=2)
        i0, j0 = rng.integers(0, n - w), rng.integers(n // 8, n - hh)
        h[j0:j0 + hh, i0:i0 + w] = rng.uniform(0.2, 1.0)
    h *= walk
    c0, c1 = int(round(0.35 * n)), int(round(0.65 * n))
    if barrier_height is not None:
        # a completed sandbag line across the inflow, two cells north of it
        jb = max(2, n // 32)
        cols = np.arange(max(c0 - n // 16, 0), min(c1 + n // 16, n))
        z[jb, cols] += barrier_height * walk[jb, cols]
    desc = I.GridDesc(nx=n, ny=n, dx=dx, dy=dx, bc=(I.WALL, I.WALL, I.WALL, I.TRANSMISSIVE),
                      inflow_side=I.SIDE_S, inflow_c0=c0, inflow_c1=c1, n_base=0.01, dt_max=dt_s)
    ht, hq = I.triangular_hydrograph(q_peak, 600.0, t_start=-float(rng.uniform(0, 300)))
    x, y = I.place_uniform(rng, walk, n_evac, dx, dx)
    agents = dict(x=x, y=y, role=np.zeros(n_evac, np.uint8), state=np.zeros(n_evac, np.uint8))
    sc = I.Scenario(desc=desc, h=h, qx=np.zeros_like(h), qy=np.zeros_like(h), z=z, hydro_t=ht, hydro_q=hq,
                    walk=walk, name=f"flood_case_{n}_{seed}")
    return FloodCase(sc=sc, agents=agents, name=sc.name)


# packed parameter layout of the library: per layer the weights
# [cout][3][3][cin] then the bias [cout]; the last layer's 3 outputs padded to 16
LAYERS = [(16, 64), (64, 64), (64, 64), (64, 64), (64, 16)]


def init_params(seed: int = 0):
    """He-normal weights (zero for the 10 unused input channels and the 13
    padding outputs) and zero biases, packed as the library expects."""
    rng = I.rng_of(seed)
    out = []
    for li, (cin, cout) in enumerate(LAYERS):
        w = rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), size=(cout, 3, 3, cin))
        if li == 0:
            w[..., N_IN:] = 0.0
        if li == len(LAYERS) - 1:
            w[3:] = 0.0
        out += [w.reshape(-1), np.zeros(cout)]
    return np.concatenate(out).astype(np.float32)


class _Crowd:
    """Device copies of a case's crowd and its per-cell counts."""

    def __init__(self, case: FloodCase, device):
        import torch
        d = case.sc.desc
        self.t = {k: torch.tensor(v, device=device).contiguous() for k, v in case.agents.items()}
        self.occ = fps.sur_occupancy(self.t["x"], self.t["y"], self.t["role"], self.t["state"],
                                     d.nx, d.ny, d.dx, d.dy)


def _flood_ensemble(cases, device="cuda"):
    ens = fps.Ensemble([c.sc for c in cases], device=device)
    crowds = [_Crowd(c, device) for c in cases]
    for m, cr in zip(ens.members, crowds):
        m.set_occupancy(cr.occ)
    return ens, crowds


def _state(m):
    return (m.h, m.qx, m.qy)


class Dataset:
    """Device-resident training pairs: x bf16 [N, n, n, 16], target fp32 [N, n, n, 4]."""

    def __init__(self, capacity, n, device="cuda"):
        import torch
        self.x = torch.empty((capacity, n, n, 16), dtype=torch.bfloat16, device=device)
        self.t = torch.empty((capacity, n, n, 4), dtype=torch.float32, device=device)
        self.n = n
        self.size = 0
        self.capacity = capacity


def generate_pairs(cases, ds: Dataset, warmup: int, pairs: int, every: int = K_STEPS, keep=None):
    """Step the cases together on the finite-volume engine and append `pairs`
    pairs per case to ds (state at t, scaled change over K steps), one every
    `every` steps after `warmup` steps.  keep: optional list collecting
    (case index, inflow feature, U0 copy, U1 copy) for evaluation.  Returns the fraction of
    pairs whose K steps all had the fixed length."""
    import torch
    ens, crowds = _flood_ensemble(cases)
    dt_s = cases[0].sc.desc.dt_max
    if warmup:
        ens.step(warmup)
    u0 = [tuple(torch.empty_like(a) for a in _state(m)) for m in ens.members]
    ok = 0
    span = K_STEPS * float(np.float32(dt_s))
    for r in range(pairs):
        t0 = [m.diag()["t"] for m in ens.members]
        feats = [m.inflow_feature(t, t + span) for m, t in zip(ens.members, t0)]
        base = ds.size
        for k, m in enumerate(ens.members):
            fps.sur_pack(m.h, m.qx, m.qy, m.z, crowds[k].occ, inflow=feats[k], out=ds.x[base + k])
            fps.sur_copy_state(_state(m), u0[k])
        ens.step(K_STEPS)
        for k, m in enumerate(ens.members):
            fps.sur_make_target(u0[k], _state(m), out=ds.t[base + k])
            if keep is not None:
                keep.append((k, feats[k], tuple(a.clone() for a in u0[k]), tuple(a.clone() for a in _state(m))))
            ok += abs(m.diag()["t"] - t0[k] - K_STEPS * float(np.float32(dt_s))) < 1e-6
        ds.size += len(cases)
        if every > K_STEPS and r + 1 < pairs:
            ens.step(every - K_STEPS)
    ens.close()
    return ok / max(1, pairs * len(cases))


def train(sur: fps.Surrogate, ds: Dataset, steps: int, batch: int, lr: float = 1e-3, lr_end: float = 5e-5,
          log_every: int = 0):
    """Adam over contiguous mini-batches of the (pre-mixed) dataset with a
    cosine learning-rate decay; returns the loss history (host floats)."""
    nb = ds.size // batch
    losses = []
    for s in range(steps):
        b = s % nb
        lr_s = lr_end + 0.5 * (lr - lr_end) * (1.0 + np.cos(np.pi * s / max(1, steps - 1)))
        loss = sur.train_step(ds.x[b * batch:(b + 1) * batch], ds.t[b * batch:(b + 1) * batch], lr_s)
        if log_every and (s % log_every == 0 or s == steps - 1):
            losses.append((s, float(loss.item())))
    return losses


def evaluate(sur: fps.Surrogate, cases, kept, tol=0.01, h_dry=1e-5):
    """Judge each held-out pair's surrogate update against the finite-volume
    one at every person's cell, beside the persistence baseline (state at t
    taken for the state at t + K steps)."""
    import torch
    n = cases[0].sc.desc.nx
    d = cases[0].sc.desc
    crowds = [_Crowd(c, "cuda") for c in cases]
    x = torch.empty((1, n, n, 16), dtype=torch.bfloat16, device="cuda")
    y = torch.empty((1, n, n, 4), dtype=torch.float32, device="cuda")
    res = {"pairs": 0, "sur_accept": 0, "persist_accept": 0, "sur_max_dh": 0.0, "persist_max_dh": 0.0,
           "sur_bad_people": 0, "persist_bad_people": 0, "people": 0, "sur_rmse_h": 0.0, "persist_rmse_h": 0.0}
    se_s = se_p = 0.0
    cells = 0
    for k, feat, u0, u1 in kept:
        cr = crowds[k].t
        z = torch.tensor(np.asarray(cases[k].sc.z, np.float32), device="cuda")
        fps.sur_pack(*u0, z, crowds[k].occ, inflow=feat, out=x[0])
        sur.forward(x, y)
        us = tuple(a.clone() for a in u0)
        fps.sur_apply(y[0], *us, h_dry=h_dry, h_snap=H_SNAP)
        js = fps.judge_result(fps.sur_judge(cr["x"], cr["y"], cr["state"], d.nx, d.ny, d.dx, d.dy, us, u1, tol=tol))
        jp = fps.judge_result(fps.sur_judge(cr["x"], cr["y"], cr["state"], d.nx, d.ny, d.dx, d.dy, u0, u1, tol=tol))
        res["pairs"] += 1
        res["people"] += len(cases[k].agents["x"])
        res["sur_accept"] += js[0] == 0
        res["persist_accept"] += jp[0] == 0
        res["sur_bad_people"] += js[0]
        res["persist_bad_people"] += jp[0]
        res["sur_max_dh"] = max(res["sur_max_dh"], js[1])
        res["persist_max_dh"] = max(res["persist_max_dh"], jp[1])
        se_s += float(((us[0] - u1[0]) ** 2).sum())
        se_p += float(((u0[0] - u1[0]) ** 2).sum())
        cells += u1[0].numel()
    res["sur_rmse_h"] = (se_s / max(cells, 1)) ** 0.5
    res["persist_rmse_h"] = (se_p / max(cells, 1)) ** 0.5
    return res


class AssistedEnsemble:
    """Surrogate-assisted flood ensemble with the finite-volume judge and
    fallback (see the module docstring).  All cases share one grid size.
    stride: every stride-th person of each crowd is a judge point."""

    def __init__(self, cases, params, chunk: int, stride: int = 1, tol: float = 0.01, halo: int = K_STEPS):
        """params: packed FP32 parameters of a trained network (any grid size)."""
        import torch
        self.torch = torch
        d0 = cases[0].sc.desc
        self.sur = fps.Surrogate(chunk, d0.ny, d0.nx)
        self.sur.set_params(params)
        self.cases, self.chunk = cases, chunk
        self.stride, self.tol = stride, tol
        d = cases[0].sc.desc
        assert all(c.sc.desc.nx == d.nx and c.sc.desc.ny == d.ny for c in cases)
        self.d = d
        self.dt = float(np.float32(d.dt_max))
        self.E, self.crowds = _flood_ensemble(cases)
        self.J, _ = _flood_ensemble(cases)
        self.masks = []
        for m, cr in zip(self.J.members, self.crowds):
            mk = fps.sur_judge_mask(cr.t["x"], cr.t["y"], cr.t["state"], d.nx, d.ny, d.dx, d.dy, halo,
                                    JUDGE_BLOCK, stride=stride)
            m.set_judge_region(mk, JUDGE_BLOCK)
            self.masks.append(mk)
        self.us = [tuple(torch.empty_like(a) for a in _state(m)) for m in self.E.members]
        self.x = torch.empty((chunk, d.ny, d.nx, 16), dtype=torch.bfloat16, device="cuda")
        self.y = torch.empty((chunk, d.ny, d.nx, 4), dtype=torch.float32, device="cuda")
        self.jout = torch.empty((len(cases), 2), dtype=torch.int32, device="cuda")
        self.t = [0.0] * len(cases)
        self.stats = {"blocks": 0, "accepted": 0, "fallback": 0, "judged_fraction": self.judged_fraction()}

    def judged_fraction(self):
        m = self.torch.stack([mk.float().mean() for mk in self.masks])
        return float(m.mean())

    def block(self):
        """Advance every case by K fixed steps; returns the accept flags."""
        S = len(self.cases)
        E, J = self.E.members, self.J.members
        # 1. the network's proposal for every case, in chunks
        span = K_STEPS * self.dt
        for c0 in range(0, S, self.chunk):
            cnt = min(self.chunk, S - c0)
            for k in range(c0, c0 + cnt):
                m = E[k]
                fps.sur_pack(m.h, m.qx, m.qy, m.z, self.crowds[k].occ,
                             inflow=m.inflow_feature(self.t[k], self.t[k] + span), out=self.x[k - c0])
            self.sur.forward(self.x[:cnt], self.y[:cnt])
            for k in range(c0, c0 + cnt):
                fps.sur_copy_state(_state(E[k]), self.us[k])
                fps.sur_apply(self.y[k - c0], *self.us[k], h_dry=self.d.h_dry, h_snap=H_SNAP)
        # 2. the finite-volume judge on the judge regions
        for k in range(S):
            fps.sur_copy_state(_state(E[k]), _state(J[k]))
            J[k].rebind_fields()
        self.J.step(K_STEPS)
        for k in range(S):
            cr = self.crowds[k].t
            fps.sur_judge(cr["x"], cr["y"], cr["state"], self.d.nx, self.d.ny, self.d.dx, self.d.dy,
                          self.us[k], _state(J[k]), tol=self.tol, h_dry=self.d.h_dry, stride=self.stride,
                          out=self.jout[k])
        bad = self.jout[:, 0].cpu().numpy()
        accept = bad == 0
        # 3. commit the accepted proposals, fall back to the finite-volume
        #    update for the others
        t_acc = [self._acc_time(t) for t in self.t]
        for k in np.flatnonzero(accept):
            fps.sur_copy_state(self.us[k], _state(E[k]))
            E[k].rebind_fields()
            E[k].set_time(t_acc[k], 0)
        rejected = np.flatnonzero(~accept)
        if len(rejected):
            for k in np.flatnonzero(accept):
                E[k].set_end_time(t_acc[k])                    # inactive while the others catch up
            for k in rejected:
                E[k].set_end_time(self.t[k] + (K_STEPS - 0.5) * self.dt)
            self.E.step(K_STEPS)
            while self.E.active() > 0:                         # a CFL-limited step made a block longer
                self.E.step(1)
            for k in range(S):
                E[k].set_end_time(0.0)
        for k in range(S):
            self.t[k] = t_acc[k] if accept[k] else E[k].diag()["t"]
            J[k].set_time(self.t[k], 0)
        self.stats["blocks"] += 1
        self.stats["accepted"] += int(accept.sum())
        self.stats["fallback"] += int((~accept).sum())
        return accept

    def _acc_time(self, t):
        """The time the engine reaches after K fixed steps from t (the same
        FP64 sums of the FP32 step)."""
        for _ in range(K_STEPS):
            t += self.dt
        return t


def timed(fn, *a, **kw):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn(*a, **kw)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0
