"""Training of the per-block damping network.

The paper damps every additive Schwarz block of a level with one factor
gamma = 1 / max_K N_K.  Here a small network maps 16 block features to
omega_j = gamma exp(clip(o_j, -3, 3)) (include/imsmg.h lists the features).

Training, all on the GPU through the library:
  1. labels: for each seeded two-level training problem (2D cubic B-splines,
     unit square minus random discs), the per-block log-weights
     theta_j = log(omega_j / gamma) minimize the two-grid objective
     J = ||E^k Z||_A^2 / ||Z||_A^2 (energy norm) of eq:eigenMulti with one
     smoothing step on each side (imsmg_two_grid_objective gives J and dJ/domega by the adjoint
     recursion); Adam on theta, clipped to [-3, 3];
  2. regression: the network is fitted to (features, theta*) with the mean
     squared error by the library's backpropagation and Adam kernels.

    python3 -m paper_1903_10977_amd.learn --problems 48 --out paper_1903_10977_amd/models/omega_mlp
    python3 -m paper_1903_10977_amd.learn --family gyroid3d --problems 64 \
        --out paper_1903_10977_amd/models/omega_mlp_gyroid3d
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import PACKAGE_DIR
from . import generator as GN
from . import solver as S

MODEL_DEFAULT = os.path.join(PACKAGE_DIR, "models", "omega_mlp")
NF, NH = 16, 64


def _log(msg):
    print(f"[learn] {msg}", file=sys.stderr, flush=True)


FAMILIES = ("discs2d", "gyroid3d")


def training_workloads(count: int, seed0: int = 10000, family: str = "discs2d"):
    """Two-level training problems.  discs2d: 2D cubic B-splines, unit square
    minus 4..12 random discs (radii U[0.03, 0.12]), 32^2 or 64^2 elements, one
    bisection level.  gyroid3d: 16^3 windows of the gyroid at the element
    size of a 96^3 grid (quadratic B-splines, random offset and phase)."""
    import workloads as W
    if family == "gyroid3d":
        return [W.gyroid_window(seed0 + i) for i in range(count)]
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        n = int(rng.choice([32, 64]))
        nd = int(rng.integers(4, 13))
        out.append(W.small_discs(seed=seed0 + i, n=n, degree=3, levels=2, n_discs=nd, depth=1,
                                 rmin=0.03, rmax=0.12, rhs="one", nu=1))
    return out


def init_params(seed: int) -> np.ndarray:
    """He-scaled normal weights, zero biases (W1, b1, W2, b2, w3, b3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.standard_normal((NH, NF)) * np.sqrt(2.0 / NF)
    W2 = rng.standard_normal((NH, NH)) * np.sqrt(2.0 / NH)
    w3 = rng.standard_normal(NH) * np.sqrt(1.0 / NH) * 0.1
    theta = np.concatenate([W1.ravel(), np.zeros(NH), W2.ravel(), np.zeros(NH), w3, np.zeros(1)])
    assert theta.size == S.MLP_PARAMS
    return theta.astype(np.float32)


def labels(sol, rng, m=8, k=8, steps=60, lr=0.05, lam_target=1.7):
    """theta* = argmin J(gamma exp(theta)) on level 1 of a two-level context,
    then shifted uniformly so that lambda_max(S A) <= lam_target (the
    stability check at inference accepts lambda_max < 1.9)."""
    n = sol._n(1)
    gamma = sol.gamma(1)
    nb = len(sol.weights(1)[0])
    Z = rng.standard_normal((n, m))
    th = np.zeros(nb)
    mo, vo = np.zeros(nb), np.zeros(nb)
    J0 = None
    for t in range(1, steps + 1):
        om = gamma * np.exp(th)
        sol.set_block_weights(1, om)
        J, g = sol.two_grid_objective(Z, k=k)
        if J0 is None:
            J0 = J
        gt = g * om  # dJ/dtheta
        mo = 0.9 * mo + 0.1 * gt
        vo = 0.999 * vo + 0.001 * gt * gt
        th -= lr * (mo / (1 - 0.9 ** t)) / (np.sqrt(vo / (1 - 0.999 ** t)) + 1e-12)
        np.clip(th, -3.0, 3.0, out=th)
    sol.set_block_weights(1, gamma * np.exp(th))
    lam = sol.lambda_max(1, 60)
    if lam > lam_target:
        th += np.log(lam_target / lam)
        sol.set_block_weights(1, gamma * np.exp(th))
    J1 = sol.two_grid_objective(Z, k=k, grad=False)
    return th, J0, J1


def train(problems=48, label_steps=60, train_steps=3000, lr=1e-3, seed=0, family="discs2d"):
    import torch
    X, T, rep = [], [], []
    for i, w in enumerate(training_workloads(problems, family=family)):
        t0 = time.time()
        g = GN.generate(w)
        sol = S.Solver(0).setup(g, S.default_options(nu_pre=1, nu_post=1)).factor()
        rng = np.random.Generator(np.random.PCG64(20000 + i))
        th, J0, J1 = labels(sol, rng, steps=label_steps)
        F = sol.features(1)
        sol.close()
        X.append(F)
        T.append(th)
        rep.append({"problem": w.name, "blocks": len(th), "J_gamma": J0, "J_labels": J1})
        _log(f"{w.name}: {len(th)} blocks, J(gamma) {J0:.4g} -> J(labels) {J1:.4g} ({time.time() - t0:.1f} s)")
    X = np.concatenate(X).astype(np.float32)
    T = np.concatenate(T).astype(np.float32)
    dev = "cuda:0"
    Xd = torch.tensor(X, device=dev)
    Td = torch.tensor(T, device=dev)
    tr = S.MlpTrainer(torch.tensor(init_params(seed), device=dev), X.shape[0])
    losses = []
    for step in range(1, train_steps + 1):
        loss = tr.step(Xd, Td, lr if step < 0.8 * train_steps else lr * 0.1)
        if step % 500 == 0 or step == 1:
            losses.append((step, float(loss.item())))
            _log(f"step {step}: loss {losses[-1][1]:.5f}")
    params = tr.params.cpu().numpy()
    o = S.mlp_forward(tr.params, Xd).cpu().numpy()
    report = {"problems": rep, "samples": int(X.shape[0]), "label_var": float(T.var()),
              "final_mse": float(np.mean((o - T) ** 2)), "losses": losses,
              "label_steps": label_steps, "train_steps": train_steps, "lr": lr, "seed": seed, "family": family}
    return params, report


def save(params, report, out=MODEL_DEFAULT):
    os.makedirs(os.path.dirname(out), exist_ok=True)
    np.save(out + ".npy", np.asarray(params, np.float32))
    with open(out + ".json", "w") as f:
        json.dump(report, f, indent=1)


def load_params(path=MODEL_DEFAULT):
    p = path + ".npy" if not path.endswith(".npy") else path
    th = np.load(p, allow_pickle=False)
    if th.shape != (S.MLP_PARAMS,):
        raise ValueError(f"{p}: expected {S.MLP_PARAMS} parameters")
    return th.astype(np.float32)


def evaluate(workloads, params, precision=S.FP64, scales=(0.8, 1.25, 1.6)):
    """PCG iterations and time with gamma, with uniformly scaled gamma (the
    tuned-scalar comparison) and with the network's weights."""
    import torch
    out = []
    for w in workloads:
        t0 = time.time()
        g = GN.generate(w)
        _log(f"{w.name}: generated {g.fine.n} DOFs in {time.time() - t0:.1f} s")
        b = torch.tensor(g.b, device="cuda:0")
        row = {"problem": w.name, "fine_dofs": int(g.fine.n), "levels": len(g.levels)}
        forms = ["gamma"] + [f"gamma x {sc}" for sc in scales] + ["learned"]
        for form in forms:
            o = S.default_options(nu_pre=w.nu, nu_post=w.nu, precision=precision, max_iter=2000,
                                  use_learned=int(form == "learned"))
            sol = S.Solver(0).setup(g, o)
            if form == "learned":
                sol.load_mlp(params)
            sol.factor()
            if form.startswith("gamma x"):
                sc = float(form.split("x")[1])
                for l in range(1, len(g.levels)):
                    sol.set_block_weights(l, sc * sol.weights(l)[0])
            x = torch.zeros_like(b)
            sol.pcg(b, x, rtol=1e-8, raise_on_error=False)  # warm-up (graph capture)
            x.zero_()
            info = sol.pcg(b, x, rtol=1e-8, raise_on_error=False)
            st = [sol.weights(l)[1] for l in range(1, len(g.levels))]
            row[form] = {"iterations": info.iterations, "ms": info.solve_ms, "true_rel_res": info.true_rel_res,
                         "status": info.status, "level_status": st}
            sol.close()
        out.append(row)
        _log(f"{w.name}: " + ", ".join(f"{f} {row[f]['iterations']} it" for f in forms) +
             f" (levels with network weights {row['learned']['level_status']})")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", type=int, default=48)
    ap.add_argument("--label-steps", type=int, default=60)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=MODEL_DEFAULT)
    ap.add_argument("--evaluate", action="store_true", help="after training, compare PCG with gamma and learned")
    ap.add_argument("--family", choices=FAMILIES, default="discs2d")
    ap.add_argument("--eval-n", type=int, nargs="*", default=None, help="evaluation grid sizes")
    a = ap.parse_args(argv)
    params, report = train(a.problems, a.label_steps, a.train_steps, a.lr, a.seed, a.family)
    if a.evaluate:
        import workloads as W
        if a.family == "gyroid3d":
            ns = a.eval_n or [48, 96]
            ws = [W.c5(n=n, levels=3 if n <= 48 else 4) for n in ns]
        else:
            ns = a.eval_n or [128, 256, 512]
            ws = [W.c2(n=n, levels=int(round(np.log2(n // 32))) + 1) for n in ns]
        report["evaluation"] = evaluate(ws, params)
    save(params, report, a.out)
    _log(f"saved {a.out}.npy (final mse {report['final_mse']:.4f}, label variance {report['label_var']:.4f})")


if __name__ == "__main__":
    main()
