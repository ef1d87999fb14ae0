"""Learned warm start of the reconstruction (Alg. 5).

A four-layer 3x3 network (64 -> 32 -> 32 -> 32 -> 64 channels, ReLU after the
first three, the last adding its input back; the q bins of an image are its
channels) works on logarithms: it maps log(x + delta) of the first EM factor
from the uniform start, x = A^T (y / (u A 1)) / b1, to an estimate o of
log(f_T / u + delta); b1 = A^T 1 is the sensitivity image and u = sum(y) /
sum(b1) the value of the plain uniform start (u x is the first unpenalised EM
iterate).  EM iterates are products of such factors, hence the log domain.
The starting image is the inverse map u max(exp(o) - delta, delta / 100),
strictly positive, scaled so that sum(b1 f0) = sum(y) (the total of every
unpenalised EM iterate; a regression on logarithms is biased low).  It is trained with Adam on pairs (log(x + delta),
log(f_T / u + delta)) where f_T is the reconstruction that Alg. 5 itself
reaches after T iterations from the uniform start.  At use, the
judge (csx_recon_warm) runs k iterations from both starts and keeps the warm
one only if its penalised objective is lower; otherwise it falls back.

Every step runs in the HIP library: convolutions on the matrix cores
(binary16 operands, float32 accumulation), loss, Adam, the input and output
maps and the solver.  This module holds device buffers and sequences calls.

    python -m paper_1603_06400_amd.warmstart --n-train 2000 --target-iters 300 --n-eval 200 --out DIR
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import csx, inputs

CHANNELS = inputs.WARM_CHANNELS
BATCH_CHUNK_MAX = 4          # scans per batch in evaluate_batched (the size every measured run used)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warm_slice128.npz")


class WarmNet:
    """Device parameters of the network (float32 master weights, binary16
    copies used by the convolutions, Adam moments, gradients)."""

    def __init__(self, params: Sequence[dict], delta: float = 0.1):
        dev = "cuda"
        self.delta = float(delta)
        self.w32 = [torch.tensor(np.asarray(p["w"], np.float32), device=dev).contiguous() for p in params]
        self.b = [torch.tensor(np.asarray(p["b"], np.float32), device=dev).contiguous() for p in params]
        self.w16 = [torch.empty(w.shape, dtype=torch.float16, device=dev) for w in self.w32]
        for w, h in zip(self.w32, self.w16):
            csx.to_half(w, h)
        self.mw = [torch.zeros_like(w) for w in self.w32]
        self.vw = [torch.zeros_like(w) for w in self.w32]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.gw = [torch.zeros_like(w) for w in self.w32]
        self.gb = [torch.zeros_like(b) for b in self.b]
        self.step_count = 0

    @classmethod
    def init(cls, seed: int, delta: float = 0.1) -> "WarmNet":
        return cls(inputs.cnn_init(seed), delta)

    @classmethod
    def load(cls, path: str = WEIGHTS) -> "WarmNet":
        with np.load(path, allow_pickle=False) as z:
            n = int(z["n_layers"])
            return cls([{"w": z[f"w{k}"], "b": z[f"b{k}"]} for k in range(n)], float(z["delta"]))

    def save(self, path: str, meta: Optional[dict] = None) -> None:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        arrs = {"n_layers": np.int64(len(self.w32)), "delta": np.float64(self.delta)}
        for k, (w, b) in enumerate(zip(self.w32, self.b)):
            arrs[f"w{k}"] = w.cpu().numpy()
            arrs[f"b{k}"] = b.cpu().numpy()
        arrs["meta"] = np.array(json.dumps(meta or {}))
        np.savez_compressed(path, **arrs)

    def layers(self):
        return list(zip(self.w16, self.b))

    def params_host(self) -> List[dict]:
        return [{"w": w.cpu().numpy(), "b": b.cpu().numpy()} for w, b in zip(self.w32, self.b)]


class Trainer:
    """Forward, backward and Adam step on minibatches of nb images h x w."""

    def __init__(self, net: WarmNet, nb: int, h: int, w: int):
        self.net, self.nb, self.h, self.w = net, nb, h, w
        dev = "cuda"
        self.acts = [torch.empty((nb, h, w, c), device=dev) for c in CHANNELS[1:]]
        self.grads = [torch.empty((nb, h, w, c), device=dev) for c in CHANNELS[1:]]
        self.ws = torch.empty(csx.cnn_workspace_bytes(nb, h, w), dtype=torch.uint8, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        src = x
        n = len(self.acts)
        for k in range(n):
            csx.conv3x3_forward(src, self.net.w16[k], self.net.b[k], self.acts[k], relu=k < n - 1,
                                residual=x if k == n - 1 else None)
            src = self.acts[k]
        return self.acts[-1]

    def backward(self, x: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
        """Loss and parameter gradients (into net.gw / net.gb) of the last forward."""
        n = len(self.acts)
        d = self.grads[-1]
        csx.warm_loss(self.acts[-1], t, d, self.loss, self.ws)
        for k in range(n - 1, -1, -1):
            inp = x if k == 0 else self.acts[k - 1]
            csx.conv3x3_backward_weights(inp, d, self.net.gw[k], self.net.gb[k], self.ws)
            if k > 0:
                csx.conv3x3_backward_data(d, self.net.w16[k], self.acts[k - 1], self.grads[k - 1])
                d = self.grads[k - 1]
        return self.loss

    def step(self, x: torch.Tensor, t: torch.Tensor, lr: float) -> torch.Tensor:
        self.forward(x)
        loss = self.backward(x, t)
        net = self.net
        net.step_count += 1
        for k in range(len(net.w32)):
            csx.adam_step(net.w32[k], net.mw[k], net.vw[k], net.gw[k], net.w16[k], net.step_count, lr)
            csx.adam_step(net.b[k], net.mb[k], net.vb[k], net.gb[k], None, net.step_count, lr)
        return loss


def counts(geo: "csx.Geometry", f_true: np.ndarray, noise_seed: int) -> torch.Tensor:
    """Poisson counts around the library's forward of f_true."""
    g = geo.forward(torch.tensor(f_true, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    return torch.tensor(inputs.poisson_counts(g, noise_seed), dtype=torch.float32, device="cuda")


def make_pairs(geo, cases, n_iter: int, beta: float, delta: float, log=None):
    """Network inputs and targets of the given cases ([n][nz][nx][nq] each)."""
    g = geo.geom
    n = len(cases)
    X = torch.empty((n, g.nz, g.nx, g.nq), device="cuda")
    T = torch.empty_like(X)
    f = geo.new_image()
    t0 = time.perf_counter()
    for i, c in enumerate(cases):
        y = counts(geo, inputs.phantom(g, c.phantom_seed, c.n_rect), c.noise_seed)
        geo.warm_input(y, delta, X[i])
        geo.recon(y, f, n_iter, beta)
        geo.warm_target(y, f, delta, T[i])
        if log and (i + 1) % 100 == 0:
            log(f"pairs {i + 1}/{n} ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    return X, T


def train(net: WarmNet, X: torch.Tensor, T: torch.Tensor, epochs: int, nb: int, lr: float, seed: int = 0,
          log=None) -> List[float]:
    """Adam over shuffled minibatches (seeded); returns the mean loss per epoch."""
    n, h, w, _ = X.shape
    tr = Trainer(net, nb, h, w)
    xb = torch.empty((nb, h, w, X.shape[3]), device="cuda")
    tb = torch.empty_like(xb)
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    for e in range(epochs):
        perm = rng.permutation(n)
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        steps = n // nb
        lr_e = lr * 0.5 * (1.0 + np.cos(np.pi * e / max(1, epochs)))    # cosine decay per epoch
        for s in range(steps):
            idx = torch.as_tensor(perm[s * nb:(s + 1) * nb], device="cuda")
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(T, 0, idx, out=tb)
            acc += tr.step(xb, tb, lr_e)
        hist.append(float(acc) / max(1, steps))
        if log:
            log(f"epoch {e + 1}/{epochs} loss {hist[-1]:.6g} lr {lr_e:.3g}")
    return hist


def first_reaching(J: np.ndarray, target: float) -> Optional[int]:
    k = np.nonzero(J <= target)[0]
    return int(k[0]) if k.size else None


def evaluate(geo, net: WarmNet, cases, n_iter: int, beta: float, k_judge: int, rel: float = 1e-3, log=None,
             os_partition=None, os_max_sweeps: int = 10):
    """Per held-out case: iterations and wall time for the plain start and for
    the judged warm start to reach J_plain(T) (1 + rel); with os_partition =
    (rho_z, rho_y) also the sweeps and wall time of ordered subsets (Alg. 6)
    from the uniform start."""
    g = geo.geom
    f = geo.new_image()
    f0 = geo.new_image()
    out = []
    for i, c in enumerate(cases):
        y = counts(geo, inputs.phantom(g, c.phantom_seed, c.n_rect), c.noise_seed)
        Jp = geo.recon(y, f, n_iter, beta)
        target = Jp[-1] + rel * abs(Jp[-1])
        n_p = first_reaching(Jp, target)
        geo.warm_start(y, net.layers(), net.delta, f0)
        Jw, acc = geo.recon_warm(y, f0, f, k_judge, n_iter, beta)
        n_w = first_reaching(Jw, target)
        # wall time to the target: plain start vs network + judge + the kept run
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        geo.recon(y, f, n_p, beta)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n_run = max(k_judge, n_w if n_w is not None else n_iter)
        geo.warm_start(y, net.layers(), net.delta, f0)
        geo.recon_warm(y, f0, f, k_judge, n_run, beta)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        row = {"case": c.phantom_seed, "J_plain_T": float(Jp[-1]), "J_warm_0": float(Jw[0]),
               "J_plain_0": float(Jp[0]), "accepted": acc, "iters_plain": n_p, "iters_warm": n_w,
               "ms_plain": (t1 - t0) * 1e3, "ms_warm": (t2 - t1) * 1e3,
               "J_warm_T": float(Jw[-1]), "J_plain": Jp.tolist(), "J_warm": Jw.tolist()}
        if os_partition is not None:
            rz, ry = os_partition
            Jo = geo.recon_os(y, f, os_max_sweeps, beta, rz, ry)
            n_o = first_reaching(Jo, target)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if n_o is not None:
                geo.recon_os(y, f, n_o, beta, rz, ry)
            torch.cuda.synchronize()
            row.update(sweeps_os=n_o, ms_os=(time.perf_counter() - t3) * 1e3 if n_o is not None else None,
                       J_os=Jo.tolist())
        out.append(row)
        if log and (i + 1) % 20 == 0:
            log(f"eval {i + 1}/{len(cases)}")
    return out


def evaluate_batched(g, net: WarmNet, cases, n_iter: int, beta: float, k_judge: int, chunk: int = 25,
                     rel: float = 1e-3, log=None) -> dict:
    """Wall time to bring every case to J_plain(n_iter) (1 + rel): the plain
    solver run case after case (each for the iterations it needs) against the
    warm path batched over `chunk` scans at a time (network per scan, the judge
    as two batched k-iteration runs, then one batched continuation in which
    each scan runs the iterations it needs).  At most BATCH_CHUNK_MAX scans
    per batch: with the batch's scans on parallel graph branches (since taken
    out), 25-scan batches ended the process with a segmentation fault whose
    cause is not found, and they stay off until it is."""
    if min(chunk, len(cases)) > BATCH_CHUNK_MAX:
        raise ValueError(f"batched warm evaluation takes at most {BATCH_CHUNK_MAX} scans per batch")
    geos = [csx.Geometry(g) for _ in range(min(chunk, len(cases)))]
    batch = csx.Batch(geos)
    t_plain = t_warm = 0.0
    accepted = 0
    iters_plain, iters_warm = [], []
    for c0 in range(0, len(cases), chunk):
        cs = cases[c0:c0 + chunk]
        if len(cs) < len(geos):
            geos_c = geos[:len(cs)]
            batch_c = csx.Batch(geos_c)
        else:
            geos_c, batch_c = geos, batch
        ys = [counts(geo, inputs.phantom(g, c.phantom_seed, c.n_rect), c.noise_seed) for geo, c in zip(geos_c, cs)]
        fp = [geo.new_image() for geo in geos_c]
        Jp = batch_c.recon(ys, fp, n_iter, beta)                       # untimed: the targets
        targets = Jp[:, -1] + rel * np.abs(Jp[:, -1])
        n_p = [first_reaching(Jp[i], targets[i]) for i in range(len(cs))]
        iters_plain += n_p
        # plain, one scan after the other, each for the iterations it needs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for geo, y, f, n in zip(geos_c, ys, fp, n_p):
            geo.recon(y, f, n, beta)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        # warm + batched: first find the iterations needed (untimed), then time the run
        fw = [geo.new_image() for geo in geos_c]
        fu = [geo.new_image() for geo in geos_c]

        def warm_run(n_cont):
            for geo, y, f in zip(geos_c, ys, fw):
                geo.warm_start(y, net.layers(), net.delta, f)
            Jw = batch_c.recon(ys, fw, k_judge, beta, init_uniform=False)
            Ju = batch_c.recon(ys, fu, k_judge, beta, init_uniform=True)
            take = Jw[:, -1] < Ju[:, -1]
            for i in range(len(cs)):
                if not take[i]:
                    fw[i].copy_(fu[i])
            Jc = batch_c.recon(ys, fw, n_cont, beta, init_uniform=False)
            J = np.concatenate([np.where(take[:, None], Jw, Ju)[:, :k_judge], Jc], axis=1)
            return J, take

        J, take = warm_run(n_iter - k_judge)
        n_w = [first_reaching(J[i], targets[i]) for i in range(len(cs))]
        n_w = [n_iter if n is None else n for n in n_w]
        iters_warm += n_w
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        warm_run([max(0, n - k_judge) for n in n_w])
        torch.cuda.synchronize()
        t_warm += time.perf_counter() - t0
        accepted += int(np.sum(take))
        if log:
            log(f"batched eval {c0 + len(cs)}/{len(cases)}")
    return {"cases": len(cases), "chunk": chunk, "k_judge": k_judge, "rel": rel,
            "total_s_plain_sequential": t_plain, "total_s_warm_batched": t_warm,
            "speedup_total": t_plain / t_warm, "accept_rate": accepted / len(cases),
            "iters_plain_mean": float(np.mean(iters_plain)), "iters_warm_mean": float(np.mean(iters_warm)),
            "iters_plain_per_case": [int(n) for n in iters_plain], "iters_warm_per_case": [int(n) for n in iters_warm]}


def summarize(rows) -> dict:
    mp = np.array([r["ms_plain"] for r in rows])
    mw = np.array([r["ms_warm"] for r in rows])
    ip = np.array([r["iters_plain"] for r in rows], dtype=float)
    iw = np.array([np.nan if r["iters_warm"] is None else r["iters_warm"] for r in rows], dtype=float)
    extra = {}
    if rows and "sweeps_os" in rows[0]:
        ok = [r for r in rows if r["sweeps_os"] is not None]
        mo = np.array([r["ms_os"] for r in ok])
        extra = {"os_reached_target": len(ok),
                 "os_sweeps_mean": float(np.mean([r["sweeps_os"] for r in ok])) if ok else None,
                 "ms_os_mean": float(mo.mean()) if ok else None,
                 "ms_os_median": float(np.median(mo)) if ok else None,
                 "speedup_os_mean_time": float(np.mean([r["ms_plain"] for r in ok]) / mo.mean()) if ok else None}
    return {**extra, "cases": len(rows), "accept_rate": float(np.mean([r["accepted"] for r in rows])),
            "ms_plain_mean": float(mp.mean()), "ms_warm_mean": float(mw.mean()),
            "ms_plain_median": float(np.median(mp)), "ms_warm_median": float(np.median(mw)),
            "s_plain_total": float(mp.sum() / 1e3), "s_warm_total": float(mw.sum() / 1e3),
            "speedup_mean_time": float(mp.mean() / mw.mean()),
            "iters_plain_mean": float(np.nanmean(ip)), "iters_warm_mean": float(np.nanmean(iw)),
            "warm_reached_target": int(np.sum(~np.isnan(iw))),
            "warm_lower_final_J": int(sum(r["J_warm_T"] <= r["J_plain_T"] for r in rows))}


def calibrated_geometry():
    """The 128^2 x 64q workload geometry with the count scale of its stored data
    (C such that the reference phantom's largest mean count is 1e4)."""
    w = inputs.workload("slice128")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    z = np.load(os.path.join(root, "tests", "golden", "slice128_counts.npz"))
    return w, w.geom.with_(C=float(z["C"]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-eval", type=int, default=200)
    ap.add_argument("--iters", type=int, default=50, help="plain iterations whose objective is the target")
    ap.add_argument("--target-iters", type=int, default=0,
                    help="iterations of the reconstructions the network is trained on (default: --iters)")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--k-judge", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--delta", type=float, default=0.1)
    ap.add_argument("--weights", default=None, help="evaluate this trained network instead of training")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    os.makedirs(args.out, exist_ok=True)
    torch.cuda.set_device(0)
    w, g = calibrated_geometry()
    geo = csx.Geometry(g)
    if args.weights:
        net = WarmNet.load(args.weights)
        with np.load(args.weights, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
        t_pairs = t_train = 0.0
    else:
        t0 = time.perf_counter()
        t_iters = args.target_iters or args.iters
        X, T = make_pairs(geo, inputs.warm_cases("train", args.n_train), t_iters, w.beta, args.delta, log)
        t_pairs = time.perf_counter() - t0
        net = WarmNet.init(args.seed, args.delta)
        t0 = time.perf_counter()
        hist = train(net, X, T, args.epochs, args.batch, args.lr, seed=args.seed, log=log)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del X, T
        meta = {"n_train": args.n_train, "iters": args.iters, "target_iters": t_iters, "epochs": args.epochs,
                "batch": args.batch,
                "lr": args.lr, "seed": args.seed, "loss": hist, "beta": w.beta, "delta": args.delta}
        net.save(os.path.join(args.out, "warm_slice128.npz"), meta)
    rows = evaluate(geo, net, inputs.warm_cases("eval", args.n_eval), args.iters, w.beta, args.k_judge, log=log)
    summ = summarize(rows)
    summ.update(seconds_pairs=t_pairs, seconds_train=t_train, k_judge=args.k_judge, rel=1e-3)
    with open(os.path.join(args.out, "warm_eval.json"), "w") as fh:
        json.dump({"summary": summ, "meta": meta, "rows": rows}, fh, indent=1)
    log(json.dumps(summ))


if __name__ == "__main__":
    sys.exit(main())
