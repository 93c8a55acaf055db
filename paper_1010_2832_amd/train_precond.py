"""Train the learned preconditioner on the method's own solves.

    python -m paper_1010_2832_amd.train_precond --out weights.npy \
        [--sizes 64,72,...,128] [--problems 286] [--chunk 48] [--epochs 3] \
        [--steps-per-chunk 1500] [--batch 8] [--init start.npy]

Problems are seeded 3D pools with spheres and a moving solid (the 256^3
benchmark family at smaller n, generator `cases.pool3d`, sizes cycled from
--sizes); pairs (r_k, e_k) come from k-iteration Jacobi-PCG iterates of each
problem (see learned.make_pairs), one pair per k in --ks.  The problems are
taken in chunks of --chunk: a chunk's contexts and pairs live on the GPU while
Adam runs --steps-per-chunk steps on random batches of its pairs, then they
are freed, so the pair set is not bounded by device memory.  Each epoch visits
every chunk; the learning rate decays geometrically from --lr to --lr-final
over all steps.  All arithmetic runs in the HIP library.  The weights are
written as a float32 .npy vector in the vfs_unet_set_weights layout (after
every chunk, so an interrupted run keeps its progress).
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
    ap.add_argument("--sizes", default="64,72,80,88,96,104,112,120,128")
    ap.add_argument("--problems", type=int, default=12)
    ap.add_argument("--first", type=int, default=0, help="index of the first problem")
    ap.add_argument("--chunk", type=int, default=48, help="problems held on the GPU at once")
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--ks", default="0,2,8,32,128,512,2048")
    ap.add_argument("--steps-per-chunk", type=int, default=1000)
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
    ids = list(range(a.first, a.first + a.problems))
    chunks = [ids[i:i + a.chunk] for i in range(0, len(ids), a.chunk)]
    total_steps = a.epochs * len(chunks) * a.steps_per_chunk
    net = V.Unet()
    w0 = np.load(a.init, allow_pickle=False) if a.init else L.he_init(a.seed)
    net.vfs_unet_set_weights(w0.astype(np.float32))
    t0 = time.time()
    done_steps = 0
    n_pairs = 0
    for epoch in range(a.epochs):
        for ci, chunk in enumerate(chunks):
            probs = []
            for i in chunk:
                n = sizes[i % len(sizes)]
                c = cases.pool3d(n, seed=a.seed + i)
                ctx = V.context_from_case(c, precision=V.VFS_MIXED)
                pairs = L.make_pairs(ctx, c["dt"], ks, device="cuda")
                ctx.vfs_assemble(c["dt"])
                probs.append((ctx, pairs))
            if epoch == 0:
                n_pairs += sum(len(p) for _, p in probs)
            log(f"epoch {epoch} chunk {ci}: {len(chunk)} problems "
                f"(n {min(sizes[i % len(sizes)] for i in chunk)}-"
                f"{max(sizes[i % len(sizes)] for i in chunk)}), pairs so far {n_pairs} "
                f"({time.time() - t0:.0f} s)")
            lr0 = a.lr * (a.lr_final / a.lr) ** (done_steps / max(1, total_steps - 1))
            lr1 = a.lr * (a.lr_final / a.lr) ** ((done_steps + a.steps_per_chunk - 1) /
                                                 max(1, total_steps - 1))
            hist = L.train(net, probs, steps=a.steps_per_chunk, lr=lr0, lr_final=lr1,
                           batch=a.batch, seed=a.seed + 7919 * (epoch * len(chunks) + ci),
                           log_every=max(1, a.steps_per_chunk // 4), log=log)
            done_steps += a.steps_per_chunk
            log(f"  mean loss {np.mean(hist[:50]):.4f} -> {np.mean(hist[-50:]):.4f} "
                f"({time.time() - t0:.0f} s)")
            np.save(a.out, net.vfs_unet_get_weights())
            for ctx, _ in probs:
                ctx.close()
            del probs, hist
            import torch
            torch.cuda.empty_cache()   # the pairs' memory back to the device
    log(f"trained {done_steps} steps on {n_pairs} pairs in {time.time() - t0:.1f} s; "
        f"weights written to {a.out}")
    net.close()


if __name__ == "__main__":
    main()
