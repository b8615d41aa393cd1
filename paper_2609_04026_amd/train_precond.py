"""Train the coarse-space preconditioner network on reduced systems this
solver generates, with the library's own forward, backward and Adam kernels.

Data: holistic scenes from the seeded generator (30 to 300 cameras, point-
only and holistic mixes, seeds disjoint from the evaluation scenes).  For
each scene a few LM steps are taken with block-Jacobi PCG; at chosen steps
the damped reduced system is read at a lambda around the solver's current
one (graph, node inputs, S blocks on the graph).  Training minimises the
mean coarse loss over batches of systems (BF16 products, FP32 accumulation)
with Adam and a cosine learning-rate decay; a held-out set of systems
reports the loss and, on its smaller systems, the loss's lower bound (the
sum of the 15 smallest eigenvalues of each block-normalised system; the
coarse space is the 7 gauge directions plus the network's 8).

    python -m paper_2609_04026_amd.train_precond --out weights.bin
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SEED_BASE = 500000  # training scenes; evaluation scenes use the workload seeds


def scene_size(rng):
    n_cams = int(round(math.exp(rng.uniform(math.log(30), math.log(300)))))
    holistic = rng.random() < 0.7
    ppc = int(rng.integers(25, 60))
    K = int(min(n_cams - 1, rng.integers(8, 33)))
    if not holistic:
        return dict(n_cams=n_cams, half=(5.0, 5.0, 2.5), radius=float(rng.uniform(12, 20)), K=K,
                    n_free_points=ppc * n_cams, n_free_lines=0, n_free_vp_lines=0, n_planes=0, n_plane_points=0,
                    n_plane_lines=0, plane_line_axis_frac=0.0, n_grids=0, grid=0, n_vps=0,
                    rot_deg=float(rng.uniform(0.5, 2.0)), trans=float(rng.uniform(0.02, 0.1)), struct=0.1, pix=1.0,
                    outlier_frac=0.0, huber=False)
    n_planes = max(3, n_cams // 6)
    return dict(n_cams=n_cams, half=(3.0, 3.0, 3.0), radius=10.0, K=K,
                n_free_points=ppc * n_cams * 3 // 4, n_free_lines=6 * n_cams, n_free_vp_lines=3 * n_cams,
                n_planes=n_planes, n_plane_points=8 * n_cams, n_plane_lines=n_cams, plane_line_axis_frac=0.5,
                n_grids=max(1, n_planes // 2), grid=4, n_vps=int(rng.integers(3, 6)),
                rot_deg=float(rng.uniform(0.5, 2.0)), trans=float(rng.uniform(0.02, 0.1)), struct=0.1, pix=1.0,
                outlier_frac=0.0, huber=False)


def _gen(seed):
    from scenegen import make_scene
    rng = np.random.default_rng(seed)
    return make_scene(scene_size(rng), seed=seed)


def collect_systems(n_scenes, per_scene, workers, log):
    """Systems from n_scenes generated scenes (scenes generated in worker processes)."""
    from paper_2609_04026_amd.binding import BA
    from paper_2609_04026_amd.precond_data import system_from_handle
    steps = [0, 2, 5, 9, 14, 20][:per_scene]
    out = []
    rng = np.random.default_rng(7)
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")  # the workers generate scenes only and never touch the GPU
    with ctx.Pool(workers) as pool:
        for k, sc in enumerate(pool.imap(_gen, [SEED_BASE + i for i in range(n_scenes)], chunksize=1)):
            ba = BA.from_scene(sc, precision="mixed", precond="jacobi")
            done = 0
            for s in range(max(steps) + 1):
                if s in steps:
                    lam_lm, _ = ba.get_lm_state()
                    lam = float(np.clip(lam_lm * 10 ** rng.uniform(-1, 1), 1e-8, 1e2)) if s else 10 ** rng.uniform(-5, -2)
                    state = ba.get_lm_state()
                    out.append(system_from_handle(ba, lam))
                    ba.set_lm_state(*state)
                    done += 1
                ba.lm_step(pcg_tol=1e-6)
            ba.close()
            if (k + 1) % 10 == 0:
                log(f"scenes {k + 1}/{n_scenes}, systems {len(out)}, {time.perf_counter() - t0:.0f}s")
    return out


def ky_fan_bound(sysd, K=15):
    """Sum of the K smallest eigenvalues of the block-normalised S of a system
    (the loss of the best 15-dimensional coarse space)."""
    n = len(sysd["node_type"])
    nA = sysd["nA"]
    S = np.zeros((nA, nA))
    off, size = sysd["node_off"], sysd["size"]
    for i in range(n):
        o, m = off[i], size[i]
        S[o:o + m, o:o + m] = sysd["s_node"][sysd["s_node_off"][i]:sysd["s_node_off"][i] + m * m].reshape(m, m)
    for e in range(len(sysd["edge_src"])):
        i, j = sysd["edge_dst"][e], sysd["edge_src"][e]
        oi, mi, oj, mj = off[i], size[i], off[j], size[j]
        S[oi:oi + mi, oj:oj + mj] = sysd["s_edge"][sysd["s_edge_off"][e]:sysd["s_edge_off"][e] + mi * mj].reshape(mi, mj)
    Linv = np.zeros_like(S)
    for i in range(n):
        o, m = off[i], size[i]
        Linv[o:o + m, o:o + m] = np.linalg.inv(np.linalg.cholesky(S[o:o + m, o:o + m]))
    return float(np.linalg.eigvalsh(Linv @ S @ Linv.T)[:K].sum())


def init_params(camera_dof, seed):
    """Gaussian weights with variance 1 / fan-in, zero biases (the blob layout of include/ba.h)."""
    from paper_2609_04026_amd.binding import gnn_param_count
    H, NIN, EIN, T = 64, 64, 8, [camera_dof * 8, 24, 16]
    rng = np.random.default_rng(seed)
    parts = [rng.normal(size=NIN * H) / math.sqrt(NIN), np.zeros(H)]
    for _ in range(3):
        parts += [rng.normal(size=(H + EIN) * H) / math.sqrt(H + EIN), np.zeros(H),
                  rng.normal(size=H * H) / math.sqrt(H), np.zeros(H)]
    for t in T:
        parts += [rng.normal(size=H * t) / math.sqrt(H), np.zeros(t)]
    p = np.concatenate(parts).astype(np.float32)
    assert len(p) == gnn_param_count(camera_dof)
    return p


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True, help="weight blob to write (float32)")
    ap.add_argument("--scenes", type=int, default=340)
    ap.add_argument("--per-scene", type=int, default=6)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--holdout", type=float, default=0.05)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--log", default=None, help="JSON summary path")
    args = ap.parse_args()

    def log(*a):
        print("[train]", *a, flush=True)

    from paper_2609_04026_amd.binding import GNN
    from paper_2609_04026_amd.precond_data import make_batch

    t0 = time.perf_counter()
    systems = collect_systems(args.scenes, min(args.per_scene, 6), args.workers, log)
    log(f"{len(systems)} systems in {time.perf_counter() - t0:.0f}s")
    rng = np.random.default_rng(args.seed)
    perm = rng.permutation(len(systems))
    n_hold = max(4, int(args.holdout * len(systems)))
    hold = [systems[i] for i in perm[:n_hold]]
    train = [systems[i] for i in perm[n_hold:]]
    # lower bound of the loss on the smaller held-out systems (dense eigenvalues)
    small = sorted(range(len(hold)), key=lambda i: hold[i]["nA"])[:24]
    bound = [ky_fan_bound(hold[i]) for i in small]
    hold_batches = [make_batch(hold[i:i + args.batch]) for i in range(0, len(hold), args.batch)]

    net = GNN(9, "bf16")
    net.set_params(init_params(9, args.seed))

    def holdout_loss():
        tot = 0.0
        for b in hold_batches:
            _, L = net.forward(b, loss=True)
            tot += L * b.s.n_graphs
        return tot / len(hold)

    small_batch = make_batch([hold[i] for i in small])

    def small_loss():
        _, L = net.forward(small_batch, loss=True)
        return L

    hist = []
    L0 = holdout_loss()
    log(f"held-out loss at init {L0:.4f}; on the {len(small)} smallest held-out systems {small_loss():.4f} "
        f"(lower bound {np.mean(bound):.4f})")
    t1 = time.perf_counter()
    for step in range(args.steps):
        lr = args.lr * 0.5 * (1 + math.cos(math.pi * step / args.steps))
        idx = rng.choice(len(train), size=args.batch, replace=False)
        L = net.train_step(make_batch([train[i] for i in idx]), lr=lr)
        if (step + 1) % 250 == 0 or step == 0:
            Lh = holdout_loss()
            Ls = small_loss()
            hist.append(dict(step=step + 1, train=L, holdout=Lh, holdout_small=Ls))
            log(f"step {step + 1}: batch loss {L:.4f}, held-out {Lh:.4f} (small {Ls:.4f} vs bound "
                f"{np.mean(bound):.4f}), {time.perf_counter() - t1:.0f}s")
    p = net.get_params()
    with open(args.out, "wb") as f:
        f.write(p.tobytes())
    summary = dict(systems=len(systems), train=len(train), holdout=len(hold), steps=args.steps, batch=args.batch,
                   lr=args.lr, holdout_loss_init=L0, holdout_loss_final=holdout_loss(),
                   holdout_small_loss_final=small_loss(), holdout_small_lower_bound=float(np.mean(bound)),
                   history=hist,
                   data_seconds=t1 - t0, train_seconds=time.perf_counter() - t1)
    log(json.dumps({k: v for k, v in summary.items() if k != "history"}))
    if args.log:
        with open(args.log, "w") as f:
            json.dump(summary, f, indent=1)
    net.close()


if __name__ == "__main__":
    main()
