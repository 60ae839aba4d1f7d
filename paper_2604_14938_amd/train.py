"""Train the bracket network on the GPU and save its weights.

Training data: seeded synthetic fields (random bubbles with radii in
[2h, 12h] and planar interfaces with random normals, on uniform hexahedral
and jittered-BCC Voronoi meshes, and wavy liquid films of random thickness,
wave count and amplitude on Voronoi pipe meshes).  Inputs are the library's own features;
labels are its plain (full-bracket) reconstructions: u* = (s* - phi_min)/W and
the interface normal, for cells whose reconstruction ended OK.  10 % of the
cells are held out; their RMS error of u gives sigma, stored with the weights
(the bracket half-width is delta_scale * W with delta_scale = 3 sigma).

Usage: python -m paper_2604_14938_amd.train [--samples N] [--steps S] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2604_14938_amd import vofpc as V  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "bracket_mlp.npz")


def log(msg: str) -> None:
    print(f"[train] {msg}", flush=True)


def xavier(seed: int, n_params: int) -> np.ndarray:
    """Xavier-uniform weights, zero biases, in the library's parameter order."""
    rng = np.random.default_rng(seed)
    shapes = [(64, 32), (64,), (64, 64), (64,), (4, 64), (4,)]
    out = []
    for s in shapes:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            out.append(rng.uniform(-lim, lim, s).ravel())
        else:
            out.append(np.zeros(s))
    v = np.concatenate(out).astype(np.float32)
    assert v.size == n_params
    return v


def field_list(seed: int, n_fields: int):
    """(mesh kind, field kind, parameters) for each training field: of every
    six, three bubble fields on Voronoi boxes, one on hexahedra, one film on
    a pipe and one plane (alternately on the two box meshes)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_fields):
        k = i % 6
        if k == 4:
            mesh_kind, field_kind = "pipe", "film"
        elif k == 5:
            mesh_kind, field_kind = ("voronoi" if (i // 6) % 2 == 0 else "hex"), "plane"
        else:
            mesh_kind, field_kind = ("hex" if k == 2 else "voronoi"), "bubbles"
        out.append((mesh_kind, field_kind, int(rng.integers(1 << 30))))
    return out


def labelled_cells(ctx, vmesh, mesh, alpha, buf):
    """Features and labels of every OK mixed cell of one field (device tensors)."""
    dev = ctx.device
    a = torch.as_tensor(alpha, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()   # written on torch's stream; the library runs on the context's
    V.compact(ctx, vmesh, a, buf["mixed"], buf["band"], buf["counts"])
    V.features(ctx, vmesh, a, buf["mixed"], buf["counts"], buf["feat"], buf["prange"])
    V.reconstruct(ctx, vmesh, a, buf["mixed"], buf["counts"], buf["itf"])
    torch.cuda.synchronize()
    M = int(buf["counts"][0].item())
    if M == 0:
        return None
    itf = buf["itf"]
    ok = itf.status[:M] == V.CELL_OK
    pr = buf["prange"][:M]
    W = pr[:, 1]
    ok &= W > 0
    u = (itf.s[:M] - pr[:, 0]) / torch.where(W > 0, W, torch.ones_like(W))
    T = torch.stack([u, itf.n[0, :M], itf.n[1, :M], itf.n[2, :M]], 1).float()
    X = buf["feat"][:M]
    return X[ok].clone(), T[ok].clone()


def _field_alpha(m, fk: str, s: int) -> np.ndarray:
    """The alpha field of one training field on mesh m (host work only)."""
    from synth import fields, workloads
    frng = np.random.default_rng(s)
    if fk == "bubbles":
        wl = workloads.random_bubbles(m, seed=s, n_max=int(frng.integers(50, 600)), K=12, r_lo_h=2.0,
                                      r_hi_h=min(float(frng.uniform(4.0, 12.0)), 0.3 / m.h))
        return wl.alpha
    if fk == "film":
        L = 52.0 / 9.5
        return fields.film_alpha(m, 1.0, float(frng.uniform(0.05, 0.2)), float(frng.uniform(0.0, 0.5)),
                                 float(frng.integers(1, 9)), L, K=12)
    nrm = frng.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    c = float(nrm @ np.full(3, 0.5) + frng.uniform(-0.25, 0.25))
    return fields.plane_alpha(m, nrm, c, K=12)


def make_dataset(ctx, n_target: int, seed: int, max_fields: int = 1200, threads: int = 8):
    """Features and labels of the fields of `field_list`, in order, until
    n_target cells are labelled.  The alpha fields are built on a thread pool
    (their C and array work releases the interpreter lock), a window at a
    time, and labelled on the device in field order."""
    from concurrent.futures import ThreadPoolExecutor
    from synth import fields, meshes
    fields._lib()       # load the sub-sampling helper once, before the threads
    lst = field_list(seed, max_fields)
    # meshes at the first use of each (kind, size slot), in field order
    rng = np.random.default_rng(seed)
    mesh_of = {}
    for i, (mk, fk, s) in enumerate(lst):
        key = (mk, (i // 6) % 3)
        if key in mesh_of:
            continue
        if mk == "voronoi":
            mesh_of[key] = meshes.voronoi_box_mesh(int(rng.choice([24, 32, 40])), seed=s)
        elif mk == "pipe":
            mesh_of[key] = meshes.voronoi_pipe_mesh(int(rng.choice([24, 30, 36])), 1.0, 52.0 / 9.5, s)
        else:
            mesh_of[key] = meshes.hex_mesh(int(rng.choice([40, 56, 72])))
    dev_of = {}
    X_parts, T_parts = [], []
    n = 0
    kinds = {}
    with ThreadPoolExecutor(max_workers=threads) as pool:
        for w0 in range(0, len(lst), threads):
            if n >= n_target:
                break
            win = list(enumerate(lst))[w0:w0 + threads]
            alphas = list(pool.map(lambda t: _field_alpha(mesh_of[(t[1][0], (t[0] // 6) % 3)], t[1][1], t[1][2]),
                                   win))
            for (i, (mk, fk, s)), alpha in zip(win, alphas):
                if n >= n_target:
                    break
                key = (mk, (i // 6) % 3)
                m = mesh_of[key]
                if key not in dev_of:
                    N = m.n_cells
                    dev = ctx.device
                    buf = dict(mixed=torch.zeros(N, dtype=torch.int32, device=dev),
                               band=torch.zeros(N, dtype=torch.int32, device=dev),
                               counts=torch.zeros(2, dtype=torch.int32, device=dev),
                               feat=torch.zeros(N, 32, dtype=torch.float32, device=dev),
                               prange=torch.zeros(N, 2, dtype=torch.float64, device=dev),
                               itf=V.Interface.empty(N, dev))
                    dev_of[key] = (V.Mesh(ctx, m), buf)
                vm, buf = dev_of[key]
                res = labelled_cells(ctx, vm, m, alpha, buf)
                if res is None:
                    continue
                X, T = res
                X_parts.append(X)
                T_parts.append(T)
                n += X.shape[0]
                kinds[f"{mk}/{fk}"] = kinds.get(f"{mk}/{fk}", 0) + int(X.shape[0])
                if i % 10 == 0:
                    log(f"field {i}: {mk}/{fk} on {m.n_cells} cells, {X.shape[0]} labelled, total {n}")
    for vm, _ in dev_of.values():
        vm.close()
    X = torch.cat(X_parts)
    T = torch.cat(T_parts)
    return X, T, kinds


def train(samples: int, steps: int, seed: int, out: str, batch: int = 4096, lr: float = 3e-3) -> dict:
    """Build the dataset, train with Adam on a cosine schedule and save the
    weights with the held-out sigma; returns the run's summary."""
    ctx = V.Context(0, stream=torch.cuda.Stream())
    t0 = time.time()
    X, T, kinds = make_dataset(ctx, samples, seed)
    t_data = time.time() - t0
    log(f"dataset: {X.shape[0]} labelled cells in {t_data:.1f} s: {kinds}")
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=g).to(X.device)
    X, T = X[perm].contiguous(), T[perm].contiguous()
    torch.cuda.synchronize()
    nval = max(1, X.shape[0] // 10)
    Xv, Tv = X[:nval].contiguous(), T[:nval].contiguous()
    Xt, Tt = X[nval:].contiguous(), T[nval:].contiguous()
    mlp = V.Mlp(ctx, max_batch=max(batch, nval))
    mlp.set_params(xavier(seed, mlp.n_params))
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    torch.cuda.synchronize()
    hist = []
    ntr = Xt.shape[0]
    t1 = time.time()
    for it in range(steps):
        j = (it * batch) % max(1, ntr - batch)
        lr_t = lr * 0.5 * (1 + np.cos(np.pi * it / steps)) + 1e-5
        mlp.train_step(Xt[j:j + batch], Tt[j:j + batch], lr_t, loss)
        if it % 200 == 0 or it == steps - 1:
            torch.cuda.synchronize()
            hist.append((it, float(loss.item())))
            log(f"step {it}: loss {hist[-1][1]:.3e}")
    torch.cuda.synchronize()
    Yv = torch.zeros(nval, 4, dtype=torch.float32, device=X.device)
    torch.cuda.synchronize()
    mlp.forward(Xv, Yv)
    torch.cuda.synchronize()
    err = (Yv[:, 0].clamp(0, 1) - Tv[:, 0]).double()
    sigma = float(err.pow(2).mean().sqrt())
    q99 = float(err.abs().quantile(0.99)) if nval > 10 else float("nan")
    params = mlp.get_params()
    info = dict(samples=int(X.shape[0]), train=int(ntr), val=int(nval), steps=steps, batch=batch, lr=lr, seed=seed,
                labels_by_kind=kinds, dataset_seconds=t_data,
                sigma_val=sigma, abs_err_q99=q99, delta_scale=3.0 * sigma, final_loss=hist[-1][1],
                train_seconds=time.time() - t1, loss_history=hist)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    np.savez(out, params=params, sigma_val=sigma, delta_scale=3.0 * sigma, info=json.dumps(info))
    log(f"validation RMS of u: {sigma:.4e} (99% abs error {q99:.3e}); saved {out}")
    mlp.close()
    return info


def load(path: str = DEFAULT_WEIGHTS) -> tuple[np.ndarray, float, dict]:
    """(parameters, delta_scale, info) of saved weights."""
    z = np.load(path, allow_pickle=False)
    return z["params"].astype(np.float32), float(z["delta_scale"]), json.loads(str(z["info"]))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=2_200_000)
    ap.add_argument("--steps", type=int, default=200000)
    ap.add_argument("--seed", type=int, default=2604)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args()
    info = train(a.samples, a.steps, a.seed, a.out)
    print(json.dumps({k: v for k, v in info.items() if k != "loss_history"}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
