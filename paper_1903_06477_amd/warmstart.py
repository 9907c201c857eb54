"""Learned warm starts for a parametric family of LASSO cone programs.

The family shares A (2000 x 1000, 2% density) and varies the data vector b
(b = A x0 + 0.05 N(0,1), x0 10%-sparse).  Any u0 is admissible for the
iteration (Sec. IV-A, equation (drs) converges from every starting point;
u0 is an input of Algorithm 1), so a network that maps b to a predicted
primal-dual triple (x, y, s) supplies u0 = (x, y + s, 1); the cold-started
method stays the fallback for every instance the warm run does not solve.

Pipeline (all on the GPU through libsscs): batched cold solves of the
training instances produce the targets; the network (2000 -> 512 -> 512 ->
10005, BF16 matrix cores, FP32 master weights, Adam, MSE on standardised
targets) is trained by the library's own kernels; input and output
standardisation are folded into the first and last layers after training, so
the deployed network maps raw b to unscaled (x, y, s).
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional

import numpy as np

from . import generators as G
from . import mlp as M
from . import sscs as S

TEST_OFFSET = 90000     # test instances are 90000.., training instances 0..


def family(indices, A=None) -> List[G.Problem]:
    if A is None:
        A = G.config5_shared_A()
    return G.config5_family(indices, A)


def features(probs) -> np.ndarray:
    return np.stack([p.meta["bd"] for p in probs]).astype(np.float32)


def solver_settings(**kw) -> S.Settings:
    base = dict(direction="aa", mem=5, eps=1e-6, lam=1.5, c1=0.9999, q=0.999, cg_tol=1e-12, cg_adapt=0.2,
                cg_max=500, max_iters=20000)
    base.update(kw)
    return S.Settings(**base)


class FamilySolver:
    """Batched solves of the shared-A family: one batch handle per chunk size
    (one device copy of A), reused for successive chunks of the family by
    replacing b and c on the device."""

    def __init__(self, settings: S.Settings, chunk: int = 10000, log=None):
        self.settings = S.Settings(**{**settings.__dict__, "data_on_device": True})
        self.chunk = chunk
        self.log = log
        self._solvers = {}

    def _solver(self, probs):
        k = len(probs)
        if k not in self._solvers:
            self._solvers[k] = [S.BatchSolver(probs, self.settings, share_A=True), None]
        return self._solvers[k]

    def solve(self, probs, u0=None):
        """Returns device tensors x (k n), y, s (k m), the infos and the
        seconds spent in the solve launches (b, c uploads excluded)."""
        import torch
        k, n, m = len(probs), probs[0].n, probs[0].m
        dev = torch.device("cuda:0")
        x = torch.empty(k * n, dtype=torch.float64, device=dev)
        y = torch.empty(k * m, dtype=torch.float64, device=dev)
        s = torch.empty(k * m, dtype=torch.float64, device=dev)
        infos, secs = [], 0.0
        N = n + m + 1
        for c0 in range(0, k, self.chunk):
            part = probs[c0:c0 + self.chunk]
            kk = len(part)
            entry = self._solver(part)
            bs, names = entry
            key = (part[0].name, part[-1].name)
            if names != key:
                b = torch.from_numpy(np.concatenate([p.b for p in part])).to(dev)
                c = torch.from_numpy(np.concatenate([p.c for p in part])).to(dev)
                bs.update_bc(b, c)
                entry[1] = key
            u = None if u0 is None else u0[c0 * N:(c0 + kk) * N]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, _, inf = bs.solve(u0_packed=u, out=(x[c0 * n:(c0 + kk) * n], y[c0 * m:(c0 + kk) * m],
                                                      s[c0 * m:(c0 + kk) * m]))
            torch.cuda.synchronize()
            secs += time.perf_counter() - t0
            infos.extend(inf)
            if self.log:
                self.log(f"  solved instances {c0}..{c0 + kk - 1} ({secs:.1f}s so far)")
        return x, y, s, infos, secs

    def close(self):
        for bs, _ in self._solvers.values():
            bs.close()
        self._solvers = {}


def batched_solve(probs, settings: S.Settings, u0=None, device=True):
    """One batched launch over probs (a fresh batch handle); returns
    (x, y, s, infos, seconds).  With device=True, u0 and the outputs are
    device tensors."""
    import torch
    st = S.Settings(**{**settings.__dict__, "data_on_device": bool(device)})
    bs = S.BatchSolver(probs, st, share_A=True)
    n, m = probs[0].n, probs[0].m
    k = len(probs)
    if device:
        out = (torch.empty(k * n, dtype=torch.float64, device="cuda:0"),
               torch.empty(k * m, dtype=torch.float64, device="cuda:0"),
               torch.empty(k * m, dtype=torch.float64, device="cuda:0"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, y, s, infos = bs.solve(u0_packed=u0, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    else:
        t0 = time.perf_counter()
        x, y, s, infos = bs.solve(u0_packed=u0)
        dt = time.perf_counter() - t0
    bs.close()
    return x, y, s, infos, dt


def family_residuals(probs, x, y, s) -> np.ndarray:
    """pr, dr, gap (Sec. IV-C) of every instance of a shared-A chunk,
    recomputed on the host in FP64 (one sparse-dense product per term)."""
    A = probs[0].A
    k, n, m = len(probs), probs[0].n, probs[0].m
    X = np.asarray(x, np.float64).reshape(k, n).T
    Y = np.asarray(y, np.float64).reshape(k, m).T
    Sv = np.asarray(s, np.float64).reshape(k, m).T
    B = np.stack([p.b for p in probs], axis=1)
    C = np.stack([p.c for p in probs], axis=1)
    nb, nc = np.linalg.norm(B, axis=0), np.linalg.norm(C, axis=0)
    pr = np.linalg.norm(A @ X + Sv - B, axis=0) / (1 + nb)
    dr = np.linalg.norm(A.T @ Y + C, axis=0) / (1 + nc)
    cx, by = np.sum(C * X, axis=0), np.sum(B * Y, axis=0)
    gap = np.abs(cx + by) / (1 + np.abs(cx) + np.abs(by))
    return np.stack([pr, dr, gap], axis=1)


class WarmStarter:
    def __init__(self, n_in: int, n_out: int, hidden=(512, 512), max_batch=1024, seed=0):
        self.widths = [n_in, *hidden, n_out]
        self.max_batch = max_batch
        self.net = M.MLP(self.widths, max_batch, seed=seed)
        self.losses: List[float] = []

    def fit(self, X: np.ndarray, T: np.ndarray, epochs=60, batch=1024, lr=1e-3, seed=0) -> List[float]:
        """Trains on standardised inputs and targets, then folds the
        standardisation into the first and last layers.  The training
        instances are independent draws, so each minibatch is a contiguous
        slice of them; every epoch visits the slices in a fresh random order."""
        import torch
        xm, xs = X.mean(0), X.std(0) + 1e-6
        tm, ts = T.mean(0), T.std(0) + 1e-6
        self.t_mean, self.t_std = tm, ts
        Xd = torch.from_numpy(((X - xm) / xs).astype(np.float32)).cuda()
        Td = torch.from_numpy(((T - tm) / ts).astype(np.float32)).cuda()
        rng = np.random.default_rng(seed)
        k = X.shape[0]
        starts = np.arange(0, k, batch)
        for ep in range(epochs):
            tot = 0.0
            for s0 in rng.permutation(starts):
                s1 = min(k, s0 + batch)
                tot += self.net.train_step(Xd[s0:s1], Td[s0:s1], lr) * (s1 - s0)
            self.losses.append(tot / k)
        Ws, bs = self.net.get_params()
        Ws = [W.astype(np.float64) for W in Ws]
        bs = [b.astype(np.float64) for b in bs]
        # first layer: W (x - xm)/xs + b = (W / xs) x + (b - W (xm / xs))
        bs[0] = bs[0] - Ws[0] @ (xm / xs)
        Ws[0] = Ws[0] / xs[None, :]
        # last layer: ts (W h + b) + tm
        Ws[-1] = Ws[-1] * ts[:, None]
        bs[-1] = bs[-1] * ts + tm
        self.net.set_params(Ws, bs)
        return self.losses

    def predict(self, Xd):
        """Predicted (x, y, s) rows for device inputs Xd (count x n_in FP32)."""
        import torch
        out = torch.empty((Xd.shape[0], self.widths[-1]), dtype=torch.float32, device=Xd.device)
        for s0 in range(0, Xd.shape[0], self.max_batch):
            s1 = min(Xd.shape[0], s0 + self.max_batch)
            self.net.forward(Xd[s0:s1], out=out[s0:s1])
        return out

    def close(self):
        self.net.close()


def targets(x, y, s, count, n, m) -> np.ndarray:
    return np.concatenate([np.asarray(x).reshape(count, n), np.asarray(y).reshape(count, m),
                           np.asarray(s).reshape(count, m)], axis=1).astype(np.float32)


def experiment(ntrain: int, ntest: int, epochs: int = 60, seed: int = 0, settings: Optional[S.Settings] = None,
               train_eps: float = 1e-4, chunk: int = 10000, log=print, lr: float = 1e-3) -> Dict:
    """Train on ntrain solved instances; test on ntest held-out instances warm
    (network inference + warm batched solve + cold fallbacks) against cold
    and against the warm start built from the training targets' mean.

    Training targets are solved to train_eps (the network's prediction error
    is far above it) and checked on the host; test instances to the
    settings' eps."""
    import torch
    st = settings or solver_settings()
    A = G.config5_shared_A()
    t0 = time.perf_counter()
    train = family(range(ntrain), A)
    test = family(range(TEST_OFFSET, TEST_OFFSET + ntest), A)
    n, m = train[0].n, train[0].m
    t_family = time.perf_counter() - t0
    log(f"family: n={n} m={m} nnz={train[0].A.nnz}, {ntrain} train / {ntest} test, generated in {t_family:.1f}s")
    # 1. training data: batched solves, checked on the host in FP64
    fs_train = FamilySolver(S.Settings(**{**st.__dict__, "eps": train_eps}), chunk, log=log)
    x, y, s, infos, t_gen = fs_train.solve(train)
    fs_train.close()
    xh, yh, sh_ = x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy()
    del x, y, s
    ok = np.array([i["status"] == S.SOLVED for i in infos])
    worst = 0.0
    for c0 in range(0, ntrain, chunk):
        c1 = min(ntrain, c0 + chunk)
        r = family_residuals(train[c0:c1], xh[c0 * n:c1 * n], yh[c0 * m:c1 * m], sh_[c0 * m:c1 * m])
        worst = max(worst, float(r[ok[c0:c1]].max()) if ok[c0:c1].any() else 0.0)
    it_train = np.array([i["iters"] for i in infos])
    log(f"training solves (eps {train_eps:g}): {t_gen:.2f}s, solved {ok.mean() * 100:.1f}%, mean "
        f"{it_train.mean():.0f} iterations, worst host-recomputed residual {worst:.2e}")
    X = features(train)[ok]
    T = targets(xh, yh, sh_, ntrain, n, m)[ok]
    del xh, yh, sh_
    # 2. train
    ws = WarmStarter(X.shape[1], T.shape[1], seed=seed)
    t1 = time.perf_counter()
    losses = ws.fit(X, T, epochs=epochs, seed=seed, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    log(f"training: {epochs} epochs in {t_train:.2f}s, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    Tmean = T.mean(0)
    del X, T
    # 3. test: cold, network warm start (+ cold fallbacks), training-mean warm start
    fs = FamilySolver(st, chunk)
    Xt = torch.from_numpy(features(test)).cuda()
    xc, yc, sc, info_cold, t_cold = fs.solve(test)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pred = ws.predict(Xt)
    u0 = M.assemble_u0(pred, n, m).reshape(-1)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t2
    xw, yw, sw, info_warm, t_warm = fs.solve(test, u0=u0)
    fail = [i for i, inf in enumerate(info_warm) if inf["status"] != S.SOLVED]
    t_fb = 0.0
    fb_solved = 0
    if fail:
        _, _, _, info_fb, t_fb = batched_solve([test[i] for i in fail], st)
        fb_solved = sum(inf["status"] == S.SOLVED for inf in info_fb)
    Tm = torch.from_numpy(np.tile(Tmean, (ntest, 1)).astype(np.float32)).cuda()
    u0m = M.assemble_u0(Tm, n, m).reshape(-1)
    del Tm
    _, _, _, info_mean, t_mean = fs.solve(test, u0=u0m)
    fs.close()
    it_mean = np.array([i["iters"] for i in info_mean])
    it_cold = np.array([i["iters"] for i in info_cold])
    it_warm = np.array([i["iters"] for i in info_warm])
    cold_ok = np.mean([i["status"] == S.SOLVED for i in info_cold])
    # held-out loss in the training standardisation (1.0 = no better than the mean)
    Tt = targets(xc.cpu().numpy(), yc.cpu().numpy(), sc.cpu().numpy(), ntest, n, m)
    test_loss = float(np.mean(((pred.cpu().numpy() - Tt) / ws.t_std) ** 2))
    del Tt
    # host check of every warm solution
    keep = np.ones(ntest, bool)
    keep[fail] = False
    rw = family_residuals(test, xw.cpu().numpy(), yw.cpu().numpy(), sw.cpu().numpy())
    wworst = float(rw[keep].max()) if keep.any() else 0.0
    ws.close()
    t_total = t_inf + t_warm + t_fb
    res = dict(ntrain=ntrain, ntest=ntest, epochs=epochs, train_eps=train_eps, t_family=t_family,
               t_generate=t_gen, iters_train_mean=float(it_train.mean()), train_worst_residual=worst,
               train_solved=float(ok.mean()), t_train=t_train,
               loss_first=losses[0], loss_last=losses[-1], t_cold=t_cold, cold_solved=float(cold_ok),
               t_inference=t_inf, t_warm_solve=t_warm, t_fallback=t_fb, n_fallback=len(fail),
               final_solved=(ntest - len(fail) + fb_solved) / ntest,
               t_warm_total=t_total, iters_cold_mean=float(it_cold.mean()),
               iters_warm_mean=float(it_warm.mean()), warm_worst_residual=wworst,
               t_mean_start=t_mean, iters_mean_start=float(it_mean.mean()), test_loss=test_loss,
               speedup=t_cold / t_total, speedup_vs_mean_start=t_mean / t_total)
    log(f"test: cold {t_cold:.2f}s ({it_cold.mean():.0f} it), warm {t_total:.2f}s = inference "
        f"{t_inf:.3f}s + solve {t_warm:.2f}s ({it_warm.mean():.0f} it) + fallback {t_fb:.2f}s ({len(fail)}); "
        f"speedup {res['speedup']:.2f}x; training-mean start {t_mean:.2f}s ({it_mean.mean():.0f} it); "
        f"held-out loss {test_loss:.3f}")
    return res


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--ntrain", type=int, default=90000)
    ap.add_argument("--ntest", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    a = ap.parse_args()
    print(json.dumps(experiment(a.ntrain, a.ntest, a.epochs, lr=a.lr, log=lambda s: print(s, flush=True))))
