"""Learned initial guess workload: 3-D Helmholtz media of random spheres
(n in [1.33, 1.5], absorbing faces ramping to kappa = 0.2, Gaussian beam on
z = 20) on a cube grid; the network (surrogate.UNet3D) is trained on
solutions of the fixed-point iteration and judged by it.

Every medium shares one canonical scaling: bias and c come from the smallest
circle holding k^2 = (k0 (n + i kappa))^2 for every n in [1.33, 1.5] and
kappa in [0, 0.2] (Sec. 3.1's construction applied to the whole range of the
media instead of one medium), so ||V|| <= 0.95 for every sample, the
symbol is shared, and the right-hand side y = -S/c (hence the scale of the
fields the network predicts) is the same for all of them.

Timed learned solve = network inference + the unchanged solver from x0, whose
first FP64 residual judges the guess: x0 is discarded for x = 0 when
||y - A x0|| >= ||y||.  Training time is reported separately.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import media, solver
from .surrogate import UNet3D, effective_parameter_count as surrogate_parameters

N_MIN, N_MAX, KAPPA_MAX = 1.33, 1.5, 0.2
WIDTH, PLANE, W0 = 16, 20, 16.0


def range_canonical(vnorm=0.95):
    """(bias, c) of the smallest circle holding k^2 over the whole (n, kappa) range; c = i R / vnorm."""
    n = np.linspace(N_MIN, N_MAX, 65)
    k = np.linspace(0.0, KAPPA_MAX, 65)
    pts = (media.K0 * (n[:, None] + 1j * k[None, :])) ** 2
    centre, R = solver.smallest_circle(pts.ravel())
    return centre, 1j * R / vnorm


class Workload:
    """Shared canonical form, absorbing layers and source for one grid shape."""

    def __init__(self, shape=(128, 128, 128), device="cuda", alpha=0.8, tol=1e-6, refine_every=20, count=200,
                 width=WIDTH, plane=PLANE, w0=W0):
        self.shape = tuple(int(s) for s in shape)
        self.device = torch.device(device)
        self.alpha, self.tol, self.k, self.count = float(alpha), float(tol), int(refine_every), int(count)
        self.bias, self.c = range_canonical()
        self.spacing = (media.H_WAVE,) * 3
        self.symbol = solver.helmholtz_symbol(self.shape, self.spacing, self.bias, self.c)
        self.kappa64 = torch.from_numpy(media.absorbing_kappa(self.shape, width, KAPPA_MAX)).to(self.device)
        self.kappa32 = self.kappa64.float()
        self.plane = min(plane, self.shape[0] - 1)
        self.w0 = float(w0)
        self.S = torch.from_numpy(media.beam_source(self.shape, self.plane, self.w0)).to(self.device)

    def features(self, net, nre):
        """Network input for one medium (the beam channels use this workload's source geometry)."""
        net.features(self.nidx(nre), plane=self.plane, w0=self.w0, k0h=media.K0 * media.H_WAVE)

    def index_maps(self, seeds):
        """Real index maps (float32 device tensors) of the seeded media, one at a time."""
        for s in seeds:
            yield torch.from_numpy(media.sphere_index(self.shape, int(s), self.count).astype(np.float32)).to(self.device)

    def nidx(self, nre):
        """Complex index n + i kappa (complex64) for the network features."""
        return torch.complex(nre, self.kappa32)

    def fields(self, nre):
        """(B, y) of the canonical system for one medium (complex128)."""
        k2 = (media.K0 * torch.complex(nre.double(), self.kappa64)) ** 2
        return solver.canonical_fields(k2, self.S, self.bias, self.c, -1.0, torch.complex128)

    def operator(self, nre, refine=True):
        B, y = self.fields(nre)
        return solver.Operator(self.symbol, B, refine=refine), y

    def solve(self, op, y, x0=None):
        return op.solve(y, x=x0, alpha=self.alpha, tol=self.tol, maxit=20000, check_every=self.k)


def make_dataset(wl: Workload, seeds, log=None):
    """Solve every seeded medium to the tolerance; returns [(nre float32, x complex64)] on the device."""
    data = []
    t0 = time.perf_counter()
    for i, nre in enumerate(wl.index_maps(seeds)):
        op, y = wl.operator(nre)
        r = wl.solve(op, y)
        if not r.converged:
            raise RuntimeError(f"training solve {i} did not converge ({r.status_name})")
        data.append((nre, r.x.to(torch.complex64)))
        op.close()
        if log and (i + 1) % 250 == 0:
            log(f"dataset {i + 1}/{len(seeds)} ({time.perf_counter() - t0:.1f} s)")
    return data


def target_scale(data):
    """RMS magnitude of the target fields (the network predicts x / scale)."""
    return float(np.sqrt(np.mean([float(x.abs().pow(2).mean()) for _, x in data])))


def train(net: UNet3D, wl: Workload, data, epochs=3, lr=2e-3, seed=0, log=None):
    """Adam, batch 1, learning rate lr * (1 + cos(pi s / steps)) / 2; returns the per-step losses."""
    rng = np.random.default_rng(seed)
    steps = max(1, epochs * len(data))
    hist = []
    # per-step losses stay on the device (no host round trip inside an epoch)
    hist_dev = torch.empty(len(data), dtype=torch.float64, device=wl.device)
    s = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        for k, j in enumerate(rng.permutation(len(data))):
            nre, x = data[j]
            wl.features(net, nre)
            net.forward()
            net.loss(x, grad=True, sync=False)
            hist_dev[k] = net.loss_device()
            net.backward()
            net.adam_step(lr=float(lr * 0.5 * (1.0 + np.cos(np.pi * s / steps))))
            s += 1
        hist.extend(hist_dev.cpu().tolist())
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {np.mean(hist[-len(data):]):.4f} "
                f"({time.perf_counter() - t0:.1f} s)")
    return hist


def _sync_time():
    torch.cuda.synchronize()
    return time.perf_counter()


def learned_solve(net: UNet3D, wl: Workload, op, y, nre, x0):
    """Inference into x0 (complex128 buffer), then the solver judging the guess: its
    first FP64 residual is that of x0, and x0 is discarded for x = 0 when
    ||y - A x0|| >= ||y||.  Returns (result, rho_x0, used)."""
    wl.features(net, nre)
    net.forward()
    net.predict_field(x0)
    r = op.solve(y, x=x0, alpha=wl.alpha, tol=wl.tol, maxit=20000, check_every=wl.k, judge_guess=True)
    rho0 = float(r.hist_true[0, 1])
    return r, rho0, bool(rho0 < 1.0)


def evaluate(net: UNet3D, wl: Workload, seeds, plain=True, log=None):
    """Per held-out medium: the solve from x0 = 0, the learned solve (inference,
    residual check, fallback, solve from x0) and, with ``plain``, the plain
    complex128 solve from 0; iterations, wall times and agreement of the solutions."""
    rows = []
    x0 = torch.empty(wl.shape, dtype=torch.complex128, device=wl.device)
    for i, nre in enumerate(wl.index_maps(seeds)):
        op, y = wl.operator(nre)
        wl.solve(op, y)                       # warm-up (first launch of this handle)
        t = _sync_time()
        r0 = wl.solve(op, y)
        t_zero = _sync_time() - t
        t = _sync_time()
        wl.features(net, nre)
        net.forward()
        net.predict_field(x0)
        t_inf = _sync_time() - t
        err0 = float((x0 - r0.x).norm() / r0.x.norm())
        t = _sync_time()
        r1, rho0, use = learned_solve(net, wl, op, y, nre, x0)
        t_learn = _sync_time() - t
        row = {"iters_zero": r0.iterations, "iters_learned": r1.iterations, "t_zero": t_zero, "t_learned": t_learn,
               "t_infer": t_inf, "rho_x0": rho0, "err_x0": err0, "used": use,
               "converged": bool(r0.converged and r1.converged),
               "diff": float((r1.x - r0.x).norm() / r0.x.norm())}
        if plain:
            opp = solver.Operator(wl.symbol, op.B, refine=False)
            wl.solve(opp, y)
            t = _sync_time()
            rp = wl.solve(opp, y)
            row["t_plain"] = _sync_time() - t
            row["iters_plain"] = rp.iterations
            row["converged"] = row["converged"] and rp.converged
            opp.close()
        op.close()
        rows.append(row)
        if log and (i + 1) % 50 == 0:
            log(f"evaluated {i + 1}/{len(seeds)}")
    return rows


def summarize(rows):
    """Means over the evaluated media (times in ms), with median and 90th percentile of
    the iteration counts and times."""
    def m(k):
        return float(np.mean([r[k] for r in rows])) if rows and k in rows[0] else None

    def q(k, scale=1.0):
        v = np.array([r[k] for r in rows], dtype=float) * scale
        return {"median": float(np.median(v)), "p90": float(np.percentile(v, 90))}

    out = {"media": len(rows), "iters_zero": m("iters_zero"), "iters_learned": m("iters_learned"),
           "t_zero_ms": 1e3 * m("t_zero"), "t_learned_ms": 1e3 * m("t_learned"), "t_infer_ms": 1e3 * m("t_infer"),
           "rho_x0": m("rho_x0"), "err_x0": m("err_x0"), "fallbacks": int(sum(not r["used"] for r in rows)),
           "all_converged": bool(all(r["converged"] for r in rows)),
           "max_solution_diff": float(max(r["diff"] for r in rows)) if rows else None}
    if rows and "t_plain" in rows[0]:
        out["t_plain_ms"] = 1e3 * m("t_plain")
        out["iters_plain"] = m("iters_plain")
    if rows:
        out["quantiles"] = {k: q(k, 1e3 if k.startswith("t_") else 1.0)
                            for k in ("iters_zero", "iters_learned", "t_zero", "t_learned", "t_plain") if k in rows[0]}
    return out


def run(shape=(128, 128, 128), n_train=2000, n_test=200, epochs=4, lr=2e-3, seed=0, plain=True, log=None, **wl_args):
    """The whole protocol: data (train seeds 0.., test seeds 10000..), training, evaluation."""
    wl = Workload(shape, **wl_args)
    t = time.perf_counter()
    data = make_dataset(wl, range(n_train), log)
    t_data = time.perf_counter() - t
    net = UNet3D(wl.shape, device=wl.device, seed=seed, scale=target_scale(data))
    t = _sync_time()
    hist = train(net, wl, data, epochs=epochs, lr=lr, seed=seed, log=log)
    t_train = _sync_time() - t
    del data
    rows = evaluate(net, wl, range(10000, 10000 + n_test), plain, log)
    res = summarize(rows)
    res.update({"grid": list(wl.shape), "train_media": n_train, "epochs": epochs, "lr": lr,
                "datagen_s": t_data, "train_s": t_train, "train_step_ms": 1e3 * t_train / max(1, len(hist)),
                "loss_first": float(np.mean(hist[:max(1, len(hist) // 20)])),
                "loss_last": float(np.mean(hist[-max(1, len(hist) // 20):])),
                "parameters": surrogate_parameters()})
    return res, net, rows
