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
* coupled_case(s): members of the large sweep (people walking to the exits)
  with the step capped at 0.01 s, for the comparison of the two arms.
* AssistedEnsemble: the surrogate-assisted coupled ensemble.  Per block of
  K steps the network proposes the next flood state of every scenario; the
  finite-volume method re-runs the K steps on the judge region only (the
  neighbourhoods of the judged people: a sample of the crowd plus everyone
  near a hazard-class boundary, see fps_set_judge_region); a scenario whose
  depth differs by more than 1 cm or whose hazard class (Table 1) differs at
  any judged person, or whose fixed step exceeds the CFL step, takes the
  coupled finite-volume steps for that block; otherwise its people walk the
  K steps on the accepted flood state.
* bar_check: every person of the plain finite-volume arm against the
  assisted arm's flood (the spec bar: 1 cm and the same class).
"""
from __future__ import annotations

import copy
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


def coupled_case(seed: int, n: int = 2048, n_evac: int = 50000, dt_s: float = 0.01, master: int = 5) -> I.Scenario:
    """A member of the large sweep (inputs.large_sweep: shopping centre with
    a completed sandbag line, the inflow under way, the free area wet, a
    crowd walking to the nearest exit) with the step capped at dt_s, so that
    K steps of the learned update span K dt_s whenever the CFL step allows."""
    sc = I._large_member((master, seed, n, n_evac))
    sc.desc.dt_max = dt_s
    return sc


def coupled_cases(S: int, n: int = 2048, n_evac: int = 50000, dt_s: float = 0.01, master: int = 5, workers: int = 8):
    """coupled_case for seeds 0 .. S-1, built in worker processes."""
    scs = I.large_sweep(S, n=n, n_evac=n_evac, seed=master, workers=workers)
    for sc in scs:
        sc.desc.dt_max = dt_s
    return scs


def _flood_only(sc: I.Scenario) -> I.Scenario:
    c = copy.copy(sc)
    c.agents = None
    c.dist = None
    c.walk = None
    c.barrier = None
    return c


class AssistedEnsemble:
    """Surrogate-assisted coupled ensemble with the finite-volume judge and
    fallback (see the module docstring).  All scenarios share one grid size.

    Per block of K steps and scenario: the network proposes the flood state
    K steps on from (h, hu, hv, z, evacuee counts); the finite-volume method
    re-runs the K steps on the judge region (the neighbourhoods of the judged
    people, with the counts of the block start); the proposal is accepted
    when every judged person's depth is within tol and hazard class is the
    same, and when the fixed step dt_max is within the CFL limit of the block
    start state.  Accepted: the flood takes the proposal and the people walk
    K steps of dt_max on it (fps_set_flood_frozen).  Rejected: K coupled
    finite-volume steps.  Judged people: every stride-th, plus everyone
    whose cell at the block start is within h_margin of the dry threshold or
    hr_margin of a Table 1 threshold."""

    def __init__(self, scenarios, params, chunk: int, stride: int = 1, tol: float = 0.01, halo: int = K_STEPS,
                 hr_margin: float = 0.1, h_margin: float = 0.01):
        import torch
        self.torch = torch
        d = scenarios[0].desc
        assert all(sc.desc.nx == d.nx and sc.desc.ny == d.ny for sc in scenarios)
        self.d, self.S, self.chunk = d, len(scenarios), chunk
        self.stride, self.tol, self.halo = stride, tol, halo
        self.hr_margin, self.h_margin = hr_margin, h_margin
        self.sur = fps.Surrogate(chunk, d.ny, d.nx)
        self.sur.set_params(params)
        self.dt = float(np.float32(d.dt_max))
        self.E = fps.Ensemble(scenarios)
        self.J = fps.Ensemble([_flood_only(sc) for sc in scenarios])
        self.us = [tuple(torch.empty_like(a) for a in _state(m)) for m in self.E.members]
        self.u0 = [tuple(torch.empty_like(a) for a in _state(m)) for m in self.E.members]
        self.x = torch.empty((chunk, d.ny, d.nx, 16), dtype=torch.bfloat16, device="cuda")
        self.y = torch.empty((chunk, d.ny, d.nx, 4), dtype=torch.float32, device="cuda")
        self.jout = torch.empty((self.S, 3), dtype=torch.int32, device="cuda")
        nb = ((d.ny + JUDGE_BLOCK - 1) // JUDGE_BLOCK, (d.nx + JUDGE_BLOCK - 1) // JUDGE_BLOCK)
        self.masks = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(self.S)]
        self.occ = [None] * self.S
        self.stats = {"blocks": 0, "accepted": 0, "fallback": 0, "cfl_fallback": 0, "judged_people": 0,
                      "judged_cells": 0.0}

    def _pick(self, k):
        a = _agents_of(self.E[k])
        return dict(stride=self.stride, select=self.u0[k], h_dry=self.d.h_dry, hr_margin=self.hr_margin,
                    h_margin=self.h_margin), a

    def block(self):
        """Advance every scenario by K steps; returns the accept flags."""
        d, S, E, J = self.d, self.S, self.E.members, self.J.members
        span = K_STEPS * self.dt
        times = [m.time() for m in E]
        cfl_ok = np.array([dtn >= self.dt for _, dtn in times])
        # 1. the network's proposal for every scenario, in chunks, from the
        #    block start state and the evacuee counts of the block start
        for k in range(S):
            fps.sur_copy_state(_state(E[k]), self.u0[k])
            self.occ[k] = E[k].counts()
        for c0 in range(0, S, self.chunk):
            cnt = min(self.chunk, S - c0)
            for k in range(c0, c0 + cnt):
                m = E[k]
                fps.sur_pack(m.h, m.qx, m.qy, m.z, self.occ[k],
                             inflow=m.inflow_feature(times[k][0], times[k][0] + span), out=self.x[k - c0])
            self.sur.forward(self.x[:cnt], self.y[:cnt])
            for k in range(c0, c0 + cnt):
                fps.sur_copy_state(self.u0[k], self.us[k])
                fps.sur_apply(self.y[k - c0], *self.us[k], h_dry=d.h_dry, h_snap=H_SNAP)
        # 2. the finite-volume judge on the judge regions of the judged people
        for k in range(S):
            pick, a = self._pick(k)
            fps.sur_judge_mask(a["x"], a["y"], a["state"], d.nx, d.ny, d.dx, d.dy, self.halo, JUDGE_BLOCK,
                               out=self.masks[k], **pick)
            J[k].set_judge_region(self.masks[k], JUDGE_BLOCK)
            fps.sur_copy_state(self.u0[k], _state(J[k]))
            J[k].rebind_fields()
            J[k].set_time(times[k][0], 0)
            J[k].set_occupancy(self.occ[k])
        self.J.step(K_STEPS)
        for k in range(S):
            pick, a = self._pick(k)
            fps.sur_judge(a["x"], a["y"], a["state"], d.nx, d.ny, d.dx, d.dy, self.us[k], _state(J[k]),
                          tol=self.tol, out=self.jout[k], **pick)
        res = self.jout.cpu().numpy()
        accept = (res[:, 0] == 0) & cfl_ok
        # 3. accepted: the proposal, and the people walk on it; rejected: the
        #    coupled finite-volume steps
        for k in np.flatnonzero(accept):
            fps.sur_copy_state(self.us[k], _state(E[k]))
            E[k].rebind_fields()
            E[k].set_flood_frozen(1)
        self.E.step(K_STEPS)
        for k in np.flatnonzero(accept):
            E[k].set_flood_frozen(0)
        self.stats["blocks"] += 1
        self.stats["accepted"] += int(accept.sum())
        self.stats["fallback"] += int((~accept).sum())
        self.stats["cfl_fallback"] += int((~cfl_ok).sum())
        self.stats["judged_people"] += int(res[:, 2].sum())
        self.stats["judged_cells"] += float(self.torch.stack([mk.float().mean() for mk in self.masks]).mean())
        return accept

    def close(self):
        self.E.close()
        self.J.close()
        self.sur.close()


def _agents_of(m):
    """The device agent arrays of a member (empty ones when it has no agents)."""
    import torch
    if getattr(m, "agents_t", None) is None:
        z = torch.zeros(0, device=m.device)
        m.agents_t = {"x": z, "y": z, "state": torch.zeros(0, dtype=torch.uint8, device=m.device)}
    return m.agents_t


def bar_check(plain, assisted: AssistedEnsemble, tol: float = 0.01):
    """Every person of the plain finite-volume ensemble (its own positions)
    against the assisted ensemble's flood: (people whose depth differs by
    more than tol or whose hazard class differs, largest depth difference)."""
    d = assisted.d
    bad, worst = 0, 0.0
    for k in range(assisted.S):
        a = _agents_of(plain[k])
        r = fps.judge_result(fps.sur_judge(a["x"], a["y"], a["state"], d.nx, d.ny, d.dx, d.dy,
                                           _state(assisted.E[k]), _state(plain[k]), tol=tol, stride=1))
        bad += r[0]
        worst = max(worst, r[1])
    return bad, worst


def timed(fn, *a, **kw):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn(*a, **kw)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0
