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
    return [G.config5_instance(int(i), A) for i in indices]


def features(probs) -> np.ndarray:
    return np.stack([p.meta["bd"] for p in probs]).astype(np.float32)


def solver_settings(**kw) -> S.Settings:
    base = dict(direction="aa", mem=5, eps=1e-6, lam=1.5, c1=0.9999, q=0.999, cg_tol=1e-12, cg_adapt=0.2,
                cg_max=500, max_iters=20000)
    base.update(kw)
    return S.Settings(**base)


def batched_solve(probs, settings: S.Settings, u0=None, device=True):
    """One persistent batched launch; returns (x, y, s, infos, seconds).
    With device=True, u0 and the outputs are device tensors."""
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


class WarmStarter:
    def __init__(self, n_in: int, n_out: int, hidden=(512, 512), max_batch=1024, seed=0):
        self.widths = [n_in, *hidden, n_out]
        self.max_batch = max_batch
        self.net = M.MLP(self.widths, max_batch, seed=seed)
        self.losses: List[float] = []

    def fit(self, X: np.ndarray, T: np.ndarray, epochs=60, batch=1024, lr=1e-3, seed=0) -> List[float]:
        """Trains on standardised inputs and targets, then folds the
        standardisation into the first and last layers."""
        import torch
        xm, xs = X.mean(0), X.std(0) + 1e-6
        tm, ts = T.mean(0), T.std(0) + 1e-6
        self.t_mean, self.t_std = tm, ts
        Xd = torch.from_numpy(((X - xm) / xs).astype(np.float32)).cuda()
        Td = torch.from_numpy(((T - tm) / ts).astype(np.float32)).cuda()
        rng = np.random.default_rng(seed)
        k = X.shape[0]
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(k)).cuda()
            tot = 0.0
            for s0 in range(0, k, batch):
                idx = perm[s0:s0 + batch]
                xb = Xd.index_select(0, idx).contiguous()
                tb = Td.index_select(0, idx).contiguous()
                tot += self.net.train_step(xb, tb, lr) * idx.numel()
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
        outs = []
        for s0 in range(0, Xd.shape[0], self.max_batch):
            outs.append(self.net.forward(Xd[s0:s0 + self.max_batch].contiguous()))
        return torch.cat(outs) if len(outs) > 1 else outs[0]


def targets(x, y, s, count, n, m) -> np.ndarray:
    return np.concatenate([np.asarray(x).reshape(count, n), np.asarray(y).reshape(count, m),
                           np.asarray(s).reshape(count, m)], axis=1).astype(np.float32)


def residuals(prob, x, y, s):
    nb, nc = np.linalg.norm(prob.b), np.linalg.norm(prob.c)
    pr = np.linalg.norm(prob.A @ x + s - prob.b) / (1 + nb)
    dr = np.linalg.norm(prob.A.T @ y + prob.c) / (1 + nc)
    cx, by = prob.c @ x, prob.b @ y
    gap = abs(cx + by) / (1 + abs(cx) + abs(by))
    return pr, dr, gap


def experiment(ntrain: int, ntest: int, epochs: int = 60, seed: int = 0, check_every: int = 1,
               settings: Optional[S.Settings] = None, log=print, lr: float = 1e-3) -> Dict:
    """Train on ntrain cold-solved instances; test on ntest instances warm
    (network inference + warm batched solve + cold fallbacks) vs cold."""
    import torch
    st = settings or solver_settings()
    A = G.config5_shared_A()
    t0 = time.perf_counter()
    train = family(range(ntrain), A)
    test = family(range(TEST_OFFSET, TEST_OFFSET + ntest), A)
    n, m = train[0].n, train[0].m
    log(f"family: n={n} m={m} nnz={train[0].A.nnz}, {ntrain} train / {ntest} test, generated in "
        f"{time.perf_counter() - t0:.1f}s")
    # 1. training data: batched cold solves, checked on the host in FP64
    x, y, s, infos, t_gen = batched_solve(train, st, device=False)
    ok = np.array([i["status"] == S.SOLVED for i in infos])
    worst = 0.0
    xs_, ys_, ss_ = x.reshape(ntrain, n), y.reshape(ntrain, m), s.reshape(ntrain, m)
    for i in range(0, ntrain, check_every):
        if ok[i]:
            worst = max(worst, max(residuals(train[i], xs_[i], ys_[i], ss_[i])))
    log(f"training solves: {t_gen:.2f}s, solved {ok.mean() * 100:.1f}%, worst host-recomputed residual {worst:.2e}")
    X = features(train)[ok]
    T = targets(x, y, s, ntrain, n, m)[ok]
    # 2. train
    ws = WarmStarter(X.shape[1], T.shape[1], seed=seed)
    t1 = time.perf_counter()
    losses = ws.fit(X, T, epochs=epochs, seed=seed, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    log(f"training: {epochs} epochs in {t_train:.2f}s, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    # 3. test: cold vs warm
    Xt = torch.from_numpy(features(test)).cuda()
    xc, yc, sc, info_cold, t_cold = batched_solve(test, st)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pred = ws.predict(Xt)
    u0 = M.assemble_u0(pred, n, m).reshape(-1)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t2
    xw, yw, sw, info_warm, t_warm = batched_solve(test, st, u0=u0)
    fail = [i for i, inf in enumerate(info_warm) if inf["status"] != S.SOLVED]
    t_fb = 0.0
    fb_solved = 0
    if fail:
        _, _, _, info_fb, t_fb = batched_solve([test[i] for i in fail], st)
        fb_solved = sum(inf["status"] == S.SOLVED for inf in info_fb)
    # ablation: the same warm start built from the training targets' mean (no network)
    Tm = torch.from_numpy(np.tile(T.mean(0), (ntest, 1)).astype(np.float32)).cuda()
    u0m = M.assemble_u0(Tm, n, m).reshape(-1)
    _, _, _, info_mean, t_mean = batched_solve(test, st, u0=u0m)
    it_mean = np.array([i["iters"] for i in info_mean])
    it_cold = np.array([i["iters"] for i in info_cold])
    # held-out loss in the training standardisation (1.0 = no better than the mean)
    Tt = targets(xc.cpu().numpy(), yc.cpu().numpy(), sc.cpu().numpy(), ntest, n, m)
    test_loss = float(np.mean(((pred.cpu().numpy() - Tt) / ws.t_std) ** 2))
    it_warm = np.array([i["iters"] for i in info_warm])
    cold_ok = np.mean([i["status"] == S.SOLVED for i in info_cold])
    # host check of the warm solutions
    xw_, yw_, sw_ = (t.cpu().numpy() for t in (xw, yw, sw))
    wworst = 0.0
    for i, p in enumerate(test):
        if i in fail:
            continue
        wworst = max(wworst, max(residuals(p, xw_[i * n:(i + 1) * n], yw_[i * m:(i + 1) * m],
                                           sw_[i * m:(i + 1) * m])))
    res = dict(ntrain=ntrain, ntest=ntest, epochs=epochs, t_generate=t_gen, t_train=t_train,
               loss_first=losses[0], loss_last=losses[-1], t_cold=t_cold, cold_solved=float(cold_ok),
               t_inference=t_inf, t_warm_solve=t_warm, t_fallback=t_fb, n_fallback=len(fail),
               final_solved=(ntest - len(fail) + fb_solved) / ntest,
               t_warm_total=t_inf + t_warm + t_fb, iters_cold_mean=float(it_cold.mean()),
               iters_warm_mean=float(it_warm.mean()), warm_worst_residual=wworst,
               t_mean_start=t_mean, iters_mean_start=float(it_mean.mean()), test_loss=test_loss,
               speedup=t_cold / (t_inf + t_warm + t_fb))
    log(f"test: cold {t_cold:.2f}s ({it_cold.mean():.0f} it), warm {t_inf + t_warm + t_fb:.2f}s = inference "
        f"{t_inf:.3f}s + solve {t_warm:.2f}s ({it_warm.mean():.0f} it) + fallback {t_fb:.2f}s ({len(fail)}); "
        f"speedup {res['speedup']:.2f}x; training-mean start {t_mean:.2f}s ({it_mean.mean():.0f} it)")
    return res


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--ntrain", type=int, default=2048)
    ap.add_argument("--ntest", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    a = ap.parse_args()
    print(json.dumps(experiment(a.ntrain, a.ntest, a.epochs, lr=a.lr, log=lambda s: print(s, flush=True))))
