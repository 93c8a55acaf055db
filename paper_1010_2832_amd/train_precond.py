"""Train the learned preconditioner on the method's own solves.

    python -m paper_1010_2832_amd.train_precond --out weights.npy \
        [--sizes 64,72,80,96] [--problems 12] [--steps 3000] [--batch 8]

Problems are seeded 3D pools with spheres and a moving solid (the 256^3
benchmark family at smaller n, generator `cases.pool3d`); pairs (r_k, e_k)
come from k-iteration Jacobi-PCG iterates of each problem (see
learned.make_pairs).  All arithmetic runs in the HIP library.  The weights
are written as a float32 .npy vector in the vfs_unet_set_weights layout.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--sizes", default="64,72,80,96")
    ap.add_argument("--problems", type=int, default=12)
    ap.add_argument("--ks", default="0,2,8,32,128,512,2048")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=5e-5)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--init", default=None, help="start from these weights (.npy)")
    a = ap.parse_args(argv)

    import cases
    from paper_1010_2832_amd import learned as L
    from paper_1010_2832_amd import vfstokes as V

    def log(m):
        print(m, flush=True)

    sizes = [int(q) for q in a.sizes.split(",")]
    ks = tuple(int(q) for q in a.ks.split(","))
    probs = []
    t0 = time.time()
    for i in range(a.problems):
        n = sizes[i % len(sizes)]
        c = cases.pool3d(n, seed=a.seed + i)
        ctx = V.context_from_case(c, precision=V.VFS_MIXED)
        pairs = L.make_pairs(ctx, c["dt"], ks, device="cuda")
        ctx.vfs_assemble(c["dt"])
        probs.append((ctx, pairs))
        log(f"problem {i}: n={n} seed={a.seed + i}, {len(pairs)} pairs ({time.time() - t0:.1f} s)")
    net = V.Unet()
    w0 = np.load(a.init, allow_pickle=False) if a.init else L.he_init(a.seed)
    net.vfs_unet_set_weights(w0.astype(np.float32))
    t0 = time.time()
    hist = L.train(net, probs, steps=a.steps, lr=a.lr, lr_final=a.lr_final, batch=a.batch,
                   seed=a.seed, log_every=250, log=log)
    log(f"trained {a.steps} steps in {time.time() - t0:.1f} s: mean loss "
        f"{np.mean(hist[:100]):.4f} -> {np.mean(hist[-100:]):.4f}")
    np.save(a.out, net.vfs_unet_get_weights())
    log(f"weights written to {a.out}")
    for ctx, _ in probs:
        ctx.close()
    net.close()


if __name__ == "__main__":
    main()
