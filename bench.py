"""Benchmark: PCG solve time per step and DOF*iter/s at 1e-6 relative residual.

Workload (default): the 2D 512^2 variable-coefficient free-surface problem
(pool of depth 0.3 + 8 seeded circles, seeded moving solid disc, smooth
log-uniform viscosity in [1, 1000], density in [0.5, 2], dt = 1e-3), solved
with mixed FP32-stencil / FP64-reduction Jacobi PCG plus FP64 iterative
refinement to 1e-6 FP64 true relative residual.  Inputs are seeded and
synthetic and resident in HBM before the timed region.

One step = reset u^n from a device copy (device-to-device), then the whole
hot path: body force, fractions, coefficients, null-space elimination,
right-hand side, PCG solve, velocity recovery.

value = sum over timed steps of (active DOFs x CG iterations) / timed wall
time, in DOF*iter/s.  The roofline object reports the dominant kernel (in
the 2D mixed inner solve the fused PCG iteration, one launch per iteration)
against MI355X HBM peak, with its average launch duration measured live by
HIP events on the context stream.

After the GPU legs, one CPU leg times the oracle (cpu_baseline) and checks
host copies of the GPU outputs against it (error_vs_fp64_oracle); nothing
else in this script runs the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(dim, precision, n_active):
    """Bytes the method must move per launch of each CG kernel.

    Per active DOF and iteration (Jacobi PCG, coefficients c per DOF: 2 in 2D
    (6 arrays over 3 unknown types), 11/6 in 3D):
      apply:  read r, D^-1, p_old and c coefficients, write p and q -> 5 + c values
      update: read x, p, r, q, D^-1, write x and r                    -> 7 values
    """
    word = 4 if precision == 1 else 8
    c = 2.0 if dim == 2 else 11.0 / 6.0
    return (5.0 + c) * word * n_active, 7.0 * word * n_active


def fused_bytes(precision, n_active):
    """Bytes one fused 2D CG iteration (one launch) must move: read r, q, p,
    D^-1, x and the c = 2 coefficients per DOF, write r, x, p, q -> 11 values
    per active DOF."""
    word = 4 if precision == 1 else 8
    return 11.0 * word * n_active


def fused3d_bytes(n_active):
    """Bytes one fused 3D CG iteration (one launch of k_fused3d, FP32) must
    move per active DOF: read r, q, p, D^-1, a, x, the sample coefficients c
    (5 per 6 samples) and face K (3 per 6 samples), write r, x, p, q -> 34/3
    values."""
    return 34.0 / 3.0 * 4 * n_active


COUNTERS = os.path.join(ROOT, "profiles", "k_fused2d_pool512_mixed_counters.md")
KERNEL_SOURCES = ("paper_1010_2832_amd/csrc/k_fused2d.hip", "paper_1010_2832_amd/csrc/vfs_reduce.h")
COUNTERS_3D = os.path.join(ROOT, "profiles", "k_fused3d_pool256_mixed_counters.md")
KERNEL_SOURCES_3D = ("paper_1010_2832_amd/csrc/k_apply3d.hip", "paper_1010_2832_amd/csrc/vfs_reduce.h",
                     "paper_1010_2832_amd/csrc/vfs_internal.h")


def _profiled_traffic(path, sources, label, row):
    """The scaled HBM bytes per launch that a committed rocprofv3 counter
    summary records in its table row `row`, or None if the summary is absent
    or the kernel sources changed since the counters were taken (SHA-256 of
    `sources` against the one recorded after `label`)."""
    import hashlib
    import re
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    m = re.search(r"sha256 \(" + re.escape(label) + r"\): ([0-9a-f]+)", text)
    t = re.search(re.escape(row) + r" \| ([0-9.eE+-]+)", text)
    if not m or not t or m.group(1) != h.hexdigest():
        return None
    return float(t.group(1))


def measured_traffic():
    """HBM bytes per launch of the fused 2D CG kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None if the kernel sources
    changed since the counters were taken (or the summary is absent)."""
    return _profiled_traffic(COUNTERS, KERNEL_SOURCES, "k_fused2d.hip + vfs_reduce.h",
                             "HBM traffic per launch (bytes, scaled)")


def measured_traffic_3d():
    """The same for the fused 3D CG kernel on the 256^3 pool."""
    return _profiled_traffic(COUNTERS_3D, KERNEL_SOURCES_3D,
                             "k_apply3d.hip + vfs_reduce.h + vfs_internal.h",
                             "HBM traffic per launch (one PCG iteration)")


def crop_errors(case, sites, got):
    """A 3D result at full size against the oracle, which cannot assemble the
    whole grid in the time of a bench run: it assembles sub-boxes of CROP^3
    cells (cases.crop) at the given sites, and at every sample and face at
    least MARGIN index steps inside one (where the oracle's values are the
    full case's) measures the GPU's active set, the residual of the GPU
    solution under the oracle's A and b (relative to the GPU's global |b|),
    and the GPU velocity against the one the oracle recovers from the GPU
    solution.  got: name -> host copies of solution and velocity (the first
    also holding rhs and active)."""
    import numpy as np
    import cases
    from cases.crop_maps import CROP, crop_lo, face_map, sample_map
    from oracle import system
    from oracle.grid import Grid
    G = Grid(case["n"], case["h"], case.get("origin"))
    first = next(iter(got.values()))
    act = np.asarray(first["active"]).astype(bool)
    nb = float(np.linalg.norm(first["rhs"][act]))
    ufl = {k: np.concatenate([G.flat(q) for q in g["velocity"]]) for k, g in got.items()}
    out = {"method": f"oracle on {CROP}^3 sub-boxes, samples at least 3 index steps inside",
           "sub_boxes": [], "active_mask_identical": True}
    worst = {k: [0.0, 0.0] for k in got}
    for label, centre in sites(case):
        lo = crop_lo(case, centre)
        C = system.assemble(cases.crop(case, lo, (CROP,) * 3))
        ci, fi = sample_map(G, C.grid, lo)
        fci, ffi = face_map(G, C.grid, lo)
        ca, fa = sample_map(G, C.grid, lo, 0)
        out["sub_boxes"].append({"site": label, "lo": list(lo),
                                 "active_compared": int(C.active[ci].sum())})
        out["active_mask_identical"] &= bool(np.array_equal(act[fi], C.active[ci]))
        live = C.K[fci] > 0
        for k, g in got.items():
            xc = np.zeros(C.grid.n_samples())
            xc[ca] = g["solution"][fa]
            r = (C.b_full - system.apply(C, xc))[ci][C.active[ci]]
            uc = system.recover_velocity(C, xc * C.active)[fci][live]
            du = np.abs(ufl[k][ffi][live] - uc).max() / max(np.abs(uc).max(), 1e-300)
            worst[k][0] = max(worst[k][0], float(np.linalg.norm(r)) / nb)
            worst[k][1] = max(worst[k][1], float(du))
    for k, (rr, du) in worst.items():
        out[k] = {"local_rel_residual_measured_by_oracle": rr,
                  "velocity_rel_linf_vs_oracle_recovery": du}
    return out


def cpu_oracle_leg(case, iters, main_out, batch_out, baseline=True, check=True, extra3d=()):
    """The CPU leg, and the only place this script runs the oracle.  It starts
    after every GPU leg has finished and reads only host copies of their
    outputs.

    cpu_baseline: the oracle as it stands assembles the explicit FP64 matrix of
    the bench workload and runs a fixed number of Jacobi-PCG iterations
    (DOF*iter/s on the host).
    error_vs_fp64_oracle: the GPU velocity, solution and active set of the
    bench workload (main_out), and of the smallest batched problem
    (batch_out), against the oracle's direct FP64 step; each 3D result in
    extra3d ((key, case, sites, host copies)) on sub-boxes (crop_errors)."""
    import numpy as np
    from oracle import cg, system
    res = {}

    def compare(c, got):
        asm, x, u = system.step(c)
        ug = np.concatenate([asm.grid.flat(q) for q in got["velocity"]])
        m = asm.K > 0
        e = {"velocity_rel_linf": float(np.abs(ug[m] - u[m]).max() / np.abs(u[m]).max()),
             "rel_residual_measured_by_oracle": float(
                 system.true_relative_residual(asm, got["solution"]))}
        if "active" in got:
            e["active_mask_identical"] = bool(np.array_equal(got["active"], asm.active))
        return e

    if check and main_out is not None:
        res["error_vs_fp64_oracle"] = compare(case, main_out)
    if check and batch_out is not None:
        e = compare(batch_out["case"], batch_out)
        res["batch64_error_vs_fp64_oracle"] = {"problem": batch_out["problem"],
                                               "n": batch_out["case"]["n"][0], **e}
    for key, c3, sites, got in extra3d:
        if check:
            res[key] = crop_errors(c3, sites, got)
    if baseline:
        t0 = time.perf_counter()
        asm = system.assemble(case)
        A, b = asm.A.tocsr(), asm.b
        t1 = time.perf_counter()
        cg.fixed_iterations(A, b, iters)
        t2 = time.perf_counter()
        n_act = A.shape[0]
        res["cpu_baseline"] = {
            "value": n_act * iters / (t2 - t1), "unit": "DOF*iter/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{case['name']} {case['n'][0]}^{len(case['n'])}: oracle assembly "
                      f"({t1 - t0:.1f} s) then {iters} Jacobi-PCG iterations on the explicit "
                      f"scipy.sparse FP64 matrix ({t2 - t1:.1f} s, single-threaded SpMV)",
            "assembly_s": t1 - t0}
    return res


WEIGHTS = os.path.join(ROOT, "paper_1010_2832_amd", "weights", "pool3d_64_96_long.npy")


def column128_leg(V):
    """FP64 plain PCG against mixed PCG with iterative refinement on the 3D
    128^3 column configuration, both to a 1e-6 FP64 relative residual.
    Returns with the figures host copies of both solutions and velocities
    (and of the right-hand side and active set) for the CPU leg to check."""
    import numpy as np
    import cases
    case = cases.column128()
    out = {"workload": "3D 128^3 column (radius 0.05, top 0.8) on a solid floor, mu 50, rho 1, "
                       "u = (0,-0.5,0), g (0,-9.8,0), dt 1e-3, seed 3, both to 1e-6"}
    vel, got = {}, {}
    for name, prec in (("fp64", V.VFS_FP64), ("mixed", V.VFS_MIXED)):
        ctx = V.context_from_case(case, precision=prec, tol=1e-6)
        ctx.vfs_set_profiling(True)
        ctx.vfs_step(case["dt"])   # first step: warms the code paths up
        ctx.vfs_set_velocity(case["u"])
        ctx.vfs_step(case["dt"])
        st = ctx.vfs_get_stats()
        got[name] = {"velocity": ctx.vfs_get_velocity(), "solution": ctx.vfs_get_solution()}
        if name == "fp64":
            got[name].update(rhs=ctx.vfs_get_rhs(), active=ctx.vfs_get_active())
        vel[name] = np.concatenate([np.ravel(q) for q in got[name]["velocity"]])
        out[name] = {"iterations": st["iterations"], "outer_iterations": st["outer_iterations"],
                     "solve_ms": st["t_solve_ms"], "step_ms": st["t_step_ms"],
                     "rel_residual_fp64": st["rel_residual"], "n_active": st["n_active"],
                     "dof_iter_per_s": st["n_active"] * st["iterations"] / (st["t_solve_ms"] * 1e-3),
                     "ms_per_iteration": st["t_solve_ms"] / max(1, st["iterations"])}
        ctx.close()
    scale = max(float(np.abs(vel["fp64"]).max()), 1e-300)
    out["velocity_rel_linf_mixed_vs_fp64"] = float(np.abs(vel["mixed"] - vel["fp64"]).max()) / scale
    return out, got


def batch64_leg(V):
    """Many uneven 2D solves in one persistent, graph-captured launch: the 64
    problems of sizes {64, 96, ..., 512}^2, tile shape and workgroups per CU
    picked by the autotuner, mixed precision to 1e-6.  Reports the solve time,
    aggregate DOF*iter/s and per-problem latency percentiles; returns with
    them host copies of the smallest problem's velocity and solution for the
    CPU leg to check."""
    import numpy as np
    import cases
    from paper_1010_2832_amd import autotune
    probs = cases.batch64()
    sizes = [c["n"][0] for c in probs]
    b = V.batch_from_cases(probs, tol=1e-6)
    b.vfs_batch_step(probs[0]["dt"])          # first step: warms the code paths up
    tune = autotune.tune(b, iterations=20, use_cache=False, cache_path=None)
    for i, c in enumerate(probs):                # the timed step starts again from u^0
        b.vfs_batch_set_problem(i, c)
    b.vfs_batch_step(probs[0]["dt"])
    st = b.vfs_batch_get_stats()
    per = [b.vfs_batch_get_problem(i) for i in range(len(probs))]
    out = {"workload": f"{len(probs)} 2D problems shaped as the 32^2 drop case, sizes "
                       f"{{64, 96, ..., 512}}^2 drawn with seed 4 ({min(sizes)}..{max(sizes)}), "
                       "mixed Jacobi PCG to 1e-6, one persistent launch per step",
           "status": st["status"], "n_problems": st["n_problems"],
           "n_active_total": st["n_active_total"], "dof_iters": st["dof_iters"],
           "solve_ms": st["t_solve_ms"], "step_ms": st["t_step_ms"],
           "dof_iter_per_s": st["dof_iters"] / (st["t_solve_ms"] * 1e-3),
           "latency_ms": {"p50": st["latency_p50_ms"], "p90": st["latency_p90_ms"],
                          "p99": st["latency_p99_ms"], "max": st["latency_max_ms"]},
           "autotune": {"shape": tune["shape"], "blocks_per_cu": tune["blocks_per_cu"],
                        "ms_per_iteration": tune["ms_per_iteration"]},
           "grid": st["grid"], "graph_used": bool(st["graph_used"]),
           "max_rel_residual_fp64": max(p["rel_residual"] for p in per),
           "max_iterations": st["max_iterations"]}
    i = int(np.argmin(sizes))
    got = {"problem": i, "case": probs[i], "velocity": b.vfs_batch_get_velocity(i),
           "solution": b.vfs_batch_get_solution(i)}
    b.close()
    return out, got


def pool256_leg(V, learned_cap=400):
    """Learned vs plain PCG on the 3D 256^3 configuration: Jacobi PCG in mixed
    precision to 1e-6, Jacobi PCG capped at learned_cap iterations, then
    truncated flexible CG with the committed network (capped at learned_cap
    iterations to bound the run) on the same step.  Returns with the figures
    host copies of the converged Jacobi-PCG solution, its velocity, the
    right-hand side and the active set for the CPU leg to check."""
    import numpy as np
    import cases
    case = cases.pool256()
    ctx = V.context_from_case(case, precision=V.VFS_MIXED, tol=1e-6)
    out = {"workload": "3D 256^3 pool (depth 0.3) + 8 spheres + moving solid sphere, mu log-uniform "
                       "[1,1000] smooth, rho [0.5,2], g (0,-9.8,0), dt 1e-3, seed 5, mixed to 1e-6"}
    ctx.vfs_set_solver(V.VFS_PRECOND_JACOBI, V.VFS_MIXED, 1e-6, 200000)
    ctx.vfs_set_profiling(True)
    ctx.vfs_step(case["dt"])
    st = ctx.vfs_get_stats()
    got = {"velocity": ctx.vfs_get_velocity(), "solution": ctx.vfs_get_solution(),
           "rhs": ctx.vfs_get_rhs(), "active": ctx.vfs_get_active()}
    out["plain_jacobi_pcg"] = {
        "iterations": st["iterations"], "solve_ms": st["t_solve_ms"], "step_ms": st["t_step_ms"],
        "rel_residual_fp64": st["rel_residual"], "n_active": st["n_active"],
        "dof_iter_per_s": st["n_active"] * st["iterations"] / (st["t_solve_ms"] * 1e-3),
        "ms_per_iteration": st["t_solve_ms"] / max(1, st["iterations"]),
        "apply_avg_ms": st["t_apply_avg_ms"], "update_avg_ms": st["t_update_avg_ms"]}
    b3, t3 = fused3d_bytes(st["n_active"]), st["t_apply_avg_ms"]
    a3 = b3 / (t3 * 1e-3) / 1e9 if t3 > 0 else 0.0
    out["plain_jacobi_pcg"]["roofline"] = {
        "bound": "hbm", "kernel": "k_fused3d (one launch per PCG iteration, FP32 vectors)",
        "achieved": a3, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a3 / HBM_PEAK_GBS,
        "traffic": measured_traffic_3d(), "avg_launch_ms": t3, "algorithmic_bytes_per_launch": b3}
    # the same step, plain PCG capped at the learned solver's iteration count
    ctx.vfs_set_solver(V.VFS_PRECOND_JACOBI, V.VFS_MIXED, 1e-6, learned_cap)
    ctx.vfs_set_velocity(case["u"])
    ctx.vfs_set_profiling(True)
    ctx.vfs_step(case["dt"], allow_unconverged=True)
    sc = ctx.vfs_get_stats()
    out["plain_jacobi_pcg_capped"] = {
        "iteration_cap": learned_cap, "iterations": sc["iterations"], "solve_ms": sc["t_solve_ms"],
        "rel_residual_fp64": sc["rel_residual"]}
    if os.path.exists(WEIGHTS):
        net = V.Unet()
        net.vfs_unet_set_weights(np.load(WEIGHTS, allow_pickle=False).astype(np.float32))
        ctx.vfs_set_preconditioner(net)
        ctx.vfs_set_solver(V.VFS_PRECOND_LEARNED, V.VFS_MIXED, 1e-6, learned_cap)
        ctx.vfs_set_velocity(case["u"])
        ctx.vfs_set_profiling(True)
        ctx.vfs_step(case["dt"], allow_unconverged=True)
        sl = ctx.vfs_get_stats()
        out["learned_fcg"] = {
            "weights": os.path.relpath(WEIGHTS, ROOT), "iteration_cap": learned_cap,
            "iterations": sl["iterations"], "solve_ms": sl["t_solve_ms"],
            "rel_residual_fp64": sl["rel_residual"], "converged": sl["rel_residual"] <= 1e-6,
            "ms_per_iteration": sl["t_solve_ms"] / max(1, sl["iterations"]),
            "precond_avg_ms": sl["t_precond_avg_ms"], "fallbacks": sl["precond_fallbacks"]}
        ctx.vfs_set_preconditioner(None)
        net.close()
    ctx.close()
    return out, got


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-check", action="store_true", help="skip the oracle comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--cpu-iters", type=int, default=3000)
    ap.add_argument("--no-column128", action="store_true",
                    help="skip the 128^3 FP64-vs-mixed leg")
    ap.add_argument("--no-batch64", action="store_true",
                    help="skip the batched 64-problem 2D leg")
    ap.add_argument("--no-pool256", action="store_true",
                    help="skip the 256^3 learned-vs-plain leg")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import cases
    from cases import crop_maps
    from paper_1010_2832_amd import vfstokes as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    case = cases.pool512(seed=args.seed, n=args.n)
    prec = V.VFS_MIXED if args.precision == "mixed" else V.VFS_FP64
    stream = torch.cuda.current_stream()

    ctx = V.context_from_case(case, precision=prec, tol=args.tol)
    ctx.vfs_set_stream(stream.cuda_stream)
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64).ravel(order="F"))).to(dev)
    u0 = [to_dev(q) for q in case["u"]]
    torch.cuda.synchronize()

    def one_step():
        ctx.vfs_set_velocity(u0)
        ctx.vfs_step(case["dt"])
        return ctx.vfs_get_stats()

    for _ in range(args.warmup):
        one_step()
    ctx.vfs_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dof_iters = 0
    iters, solve_ms, n_act, res = [], [], 0, []
    for _ in range(args.steps):
        st = one_step()
        n_act = st["n_active"]
        dof_iters += st["n_active"] * st["iterations"]
        iters.append(st["iterations"])
        solve_ms.append(st["t_solve_ms"])
        res.append(st["rel_residual"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ctx.vfs_get_stats()
    ctx.vfs_set_profiling(False)
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps

    ta, tu = st["t_apply_avg_ms"], st["t_update_avg_ms"]
    if prec == V.VFS_MIXED:
        # one fused launch per CG iteration in the 2D mixed inner solve
        dom = ("k_fused2d (one launch per PCG iteration: lazy x, r update, Jacobi, direction, "
               "matrix-free A p, five FP64 partials)")
        bytes_, t_ms = fused_bytes(prec, n_act), ta
    else:
        b_apply, b_update = algorithmic_bytes(2, prec, n_act)
        if ta * b_update / max(b_apply, 1) >= tu:
            dom, bytes_, t_ms = "k_apply2d (fused direction update + matrix-free apply + p.Ap)", b_apply, ta
        else:
            dom, bytes_, t_ms = "k_update (x, r update + Jacobi + r.z, r.r)", b_update, tu
    achieved = bytes_ / (t_ms * 1e-3) / 1e9 if t_ms > 0 else 0.0

    out = {
        "metric": "PCG solve time/step & DOF*iter/s at 1e-6 rel residual (plain Jacobi PCG)",
        "value": dof_iters / wall,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == V.VFS_MIXED else "f64",
        "data": "synthetic (seeded generator, inputs resident in HBM)",
        "config": {"workload": f"2D {args.n}^2 pool + 8 circles + moving solid disc, mu log-uniform "
                               f"[1,1000] smooth, rho [0.5,2], dt 1e-3, {args.precision} Jacobi PCG to "
                               f"{args.tol:g}",
                   "seed": args.seed, "n": args.n, "tol": args.tol, "precision": args.precision,
                   "n_active": int(n_act), "cg_iterations_per_step": iters,
                   "solve_ms_per_step": [round(s, 3) for s in solve_ms],
                   "rel_residual_fp64": res,
                   "assemble_ms": st["t_assemble_ms"], "recover_ms": st["t_recover_ms"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if (args.n == 512 and dom.startswith("k_fused2d"))
                                else None,
                     "avg_launch_ms": t_ms, "launches_timed": int(st["n_apply_timed"]),
                     "algorithmic_bytes_per_launch": bytes_,
                     "apply_avg_ms": ta, "update_avg_ms": tu},
    }
    out["paper_context"] = {
        "timings": None,
        "note": "the paper reports no wall-clock times, hardware or precision; its only solver "
                "figures are PCG iteration counts with an overlapping multiplicative Schwarz "
                "preconditioner (Table 1: 2D free-surface disk, 54 at 512^2 and 110 at 1024^2, "
                "one step with dt = 1), against Jacobi PCG here"}
    main_got = {"velocity": ctx.vfs_get_velocity(), "solution": ctx.vfs_get_solution(),
                "active": ctx.vfs_get_active()}
    ctx.close()
    batch_got, extra3d, got = None, [], None
    if not args.no_column128:
        out["column128_fp64_vs_mixed"], got = column128_leg(V)
        extra3d.append(("column128_fp64_vs_mixed", cases.column128(), crop_maps.sites_column, got))
    if not args.no_batch64:
        out["batch64_2d"], batch_got = batch64_leg(V)
    if not args.no_pool256:
        out["pool256_learned_vs_plain"], got = pool256_leg(V)
        extra3d.append(("pool256_learned_vs_plain", cases.pool256(), crop_maps.sites_pool,
                        {"plain_jacobi_pcg": got}))
    del got
    if not (args.no_check and args.no_cpu):
        res = cpu_oracle_leg(case, args.cpu_iters, main_got, batch_got,
                             baseline=not args.no_cpu, check=not args.no_check, extra3d=extra3d)
        for key in ("error_vs_fp64_oracle", "cpu_baseline"):
            if key in res:
                out[key] = res[key]
        if "batch64_error_vs_fp64_oracle" in res:
            out["batch64_2d"]["error_vs_fp64_oracle"] = res["batch64_error_vs_fp64_oracle"]
        for key, _, _, _ in extra3d:
            if key in res:
                out[key]["error_vs_fp64_oracle"] = res[key]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
