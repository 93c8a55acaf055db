"""Benchmark: PCG solve time per step and DOF*iter/s at 1e-6 relative residual;
learned vs plain PCG.

Headline workload: the 3D 256^3 variable-coefficient free-surface problem
(pool of depth 0.3 + 8 seeded spheres, seeded moving solid sphere, smooth
log-uniform viscosity in [1, 1000], density in [0.5, 2], g = (0, -9.8, 0),
dt = 1e-3), solved with plain Jacobi PCG in mixed precision (FP32 stencil and
vectors, FP64 reductions, FP64 residual and iterative refinement) to 1e-6
FP64 true relative residual.  Inputs are seeded and synthetic and resident in
HBM before the timed region.

One step = reset u^n from a device copy (device-to-device), then the whole
hot path: body force, fractions, coefficients, null-space elimination,
right-hand side, PCG solve, velocity recovery.

value = sum over timed steps of (active DOFs x CG iterations) / timed wall
time, in DOF*iter/s.  The roofline object reports the dominant kernel (the
fused 3D PCG iteration, one launch per iteration) against MI355X HBM peak:
algorithmic bytes per launch (12 + c values of 4 bytes per active DOF, c =
11/6 coefficients per DOF) over its average launch duration, measured live
by HIP events on the context stream.

Legs beside the headline: learned flexible CG on the same step (to 1e-6, or
to an iteration cap, reported as not converged), the 2D 512^2 problem, the
3D 128^3 column in FP64 and mixed precision, and the 64 batched 2D problems.
After the GPU legs, one CPU leg times the oracle on a bounded sample of the
headline workload (cpu_baseline) and checks host copies of the GPU outputs
against it (error_vs_fp64_oracle); nothing else in this script runs the
oracle.
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


def pcg_values_per_dof(dim):
    """Values the fused Jacobi PCG iteration must move per active DOF:
    direction + apply (read r, D^-1, p and the c coefficients, write p and q:
    5 + c) and the update (read x, p, r, q, D^-1, write x and r: 7), so 12 + c,
    with c = 6/3 coefficients per DOF in 2D (W_L and c per sample, K per
    face) and 11/6 in 3D."""
    return 12.0 + (2.0 if dim == 2 else 11.0 / 6.0)


def fused2d_bytes(n_active):
    """Algorithmic bytes of one fused 2D CG iteration in FP32 (56 per DOF)."""
    return pcg_values_per_dof(2) * 4 * n_active


def fused3d_bytes(n_active):
    """Algorithmic bytes of one fused 3D CG iteration in FP32 (55.3 per DOF)."""
    return pcg_values_per_dof(3) * 4 * n_active


COUNTERS_2D = os.path.join(ROOT, "profiles", "k_fused2d_pool512_mixed_counters.md")
KERNEL_SOURCES_2D = ("paper_1010_2832_amd/csrc/k_fused2d.hip", "paper_1010_2832_amd/csrc/vfs_reduce.h")
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


def measured_traffic_2d():
    """HBM bytes per launch of the fused 2D CG kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None if the kernel sources
    changed since the counters were taken (or the summary is absent)."""
    return _profiled_traffic(COUNTERS_2D, KERNEL_SOURCES_2D, "k_fused2d.hip + vfs_reduce.h",
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
    full case's) measures the GPU's active set, the residual r = b - A x of
    the GPU solution under the oracle's A and b over the compared samples --
    as a local backward error |r| / | |A| |x| + |b| | (relative to the size of
    the terms that cancel in those rows, so a sub-box where b vanishes is
    still judged) and relative to the GPU's global |b| -- and the GPU velocity
    against the one the oracle recovers from the GPU solution.  got: name -> host copies of solution and velocity
    (the first also holding rhs and active)."""
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
    worst = {k: [0.0, 0.0, 0.0] for k in got}
    for label, centre in sites(case):
        lo = crop_lo(case, centre)
        C = system.assemble(cases.crop(case, lo, (CROP,) * 3))
        ci, fi = sample_map(G, C.grid, lo)
        fci, ffi = face_map(G, C.grid, lo)
        ca, fa = sample_map(G, C.grid, lo, 0)
        absA = abs(C.A_full).tocsr()
        out["sub_boxes"].append({"site": label, "lo": list(lo),
                                 "active_compared": int(C.active[ci].sum())})
        out["active_mask_identical"] &= bool(np.array_equal(act[fi], C.active[ci]))
        live = C.K[fci] > 0
        for k, g in got.items():
            xc = np.zeros(C.grid.n_samples())
            xc[ca] = g["solution"][fa]
            sel = ci[C.active[ci]]
            r = (C.b_full - system.apply(C, xc))[sel]
            terms = (absA @ np.abs(xc * C.active) + np.abs(C.b_full))[sel]
            uc = system.recover_velocity(C, xc * C.active)[fci][live]
            du = np.abs(ufl[k][ffi][live] - uc).max() / max(np.abs(uc).max(), 1e-300)
            rn = float(np.linalg.norm(r))
            worst[k][0] = max(worst[k][0], rn / max(float(np.linalg.norm(terms)), 1e-300))
            worst[k][1] = max(worst[k][1], rn / nb)
            worst[k][2] = max(worst[k][2], float(du))
    for k, (rl, rg, du) in worst.items():
        out[k] = {"local_backward_error": rl,
                  "local_residual_vs_global_b": rg,
                  "velocity_rel_linf_vs_oracle_recovery": du}
    return out


def host_cpu():
    """Model name and logical CPU count of the host this script runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def cpu_oracle_leg(baseline_case, iters, main_out, batch_out, baseline=True, check=True,
                   extra3d=(), extra2d=()):
    """The CPU leg, and the only place this script runs the oracle.  It starts
    after every GPU leg has finished and reads only host copies of their
    outputs.

    cpu_baseline: the oracle as it stands assembles the explicit FP64 matrix of
    a bounded sample of the headline workload (a sub-box of the 256^3 pool)
    and runs a fixed number of Jacobi-PCG iterations on one thread
    (DOF*iter/s on the host).
    error_vs_fp64_oracle: each 3D result in extra3d ((key, case, sites, host
    copies)) on sub-boxes (crop_errors); each 2D result in extra2d ((key,
    case, host copies)) and the batched problems in batch_out (the smallest,
    middle and largest) against the oracle's direct FP64 step."""
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

    for key, c3, sites, got in extra3d:
        if check:
            res[key] = crop_errors(c3, sites, got)
    for key, c2, got in extra2d:
        if check:
            res[key] = compare(c2, got)
    if check and batch_out:
        res["batch64_error_vs_fp64_oracle"] = [
            {"problem": q["problem"], "n": q["case"]["n"][0], "tol": q["tol"],
             **compare(q["case"], q)} for q in batch_out]
    if baseline and baseline_case is not None:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            asm = system.assemble(baseline_case)
            A, b = asm.A.tocsr(), asm.b
            t1 = time.perf_counter()
            cg.fixed_iterations(A, b, iters)
            t2 = time.perf_counter()
        n_act = A.shape[0]
        res["cpu_baseline"] = {
            "value": n_act * iters / (t2 - t1), "unit": "DOF*iter/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{baseline_case['name']}: the oracle's assembly of this "
                      f"{baseline_case['n'][0]}^3 sub-box of the 256^3 pool ({n_act} active "
                      f"DOFs, {t1 - t0:.1f} s, not timed), then {iters} FP64 Jacobi-PCG iterations "
                      f"on its explicit scipy.sparse matrix ({t2 - t1:.1f} s, timed), one thread",
            "assembly_s": t1 - t0, **host_cpu()}
    return res


WEIGHTS = os.path.join(ROOT, "paper_1010_2832_amd", "weights", "pool3d_64_128.npy")


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


# The batched configuration leaves its tolerance unstated.  The velocity error
# against the FP64 oracle grows with the problem's conditioning: at 1e-6 the
# 64^2 problem was 1.35e-4 off and at 1e-7 the 320^2 one 4.2e-4, both above
# the mixed path's 1e-4 bar; 1e-9 keeps the smallest, middle and largest
# problems within it.
BATCH_TOL = 1e-9


def batch64_leg(V):
    """Many uneven 2D solves in one persistent, graph-captured launch: the 64
    problems of sizes {64, 96, ..., 512}^2, tile shape and workgroups per CU
    picked by the autotuner, mixed precision to BATCH_TOL.  Reports the solve time,
    aggregate DOF*iter/s and per-problem latency percentiles; returns with
    them host copies of the velocity and solution of the smallest, middle and
    largest problems for the CPU leg to check."""
    import numpy as np
    import cases
    from paper_1010_2832_amd import autotune
    probs = cases.batch64()
    sizes = [c["n"][0] for c in probs]
    b = V.batch_from_cases(probs, tol=BATCH_TOL)
    b.vfs_batch_step(probs[0]["dt"])          # first step: warms the code paths up
    tune = autotune.tune(b, iterations=20, use_cache=False, cache_path=None)
    for i, c in enumerate(probs):                # the timed step starts again from u^0
        b.vfs_batch_set_problem(i, c)
    b.vfs_batch_step(probs[0]["dt"])
    st = b.vfs_batch_get_stats()
    per = [b.vfs_batch_get_problem(i) for i in range(len(probs))]
    out = {"workload": f"{len(probs)} 2D problems shaped as the 32^2 drop case, sizes "
                       f"{{64, 96, ..., 512}}^2 drawn with seed 4 ({min(sizes)}..{max(sizes)}), "
                       f"mixed Jacobi PCG to {BATCH_TOL:g}, one persistent launch per step",
           "tol": BATCH_TOL,
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
    order = np.argsort(sizes, kind="stable")
    got = []
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        got.append({"problem": i, "case": probs[i], "tol": BATCH_TOL,
                    "velocity": b.vfs_batch_get_velocity(i), "solution": b.vfs_batch_get_solution(i)})
    b.close()
    return out, got


def timed_steps(ctx, u0, dt, steps, warmup):
    """`warmup` untimed steps, then `steps` timed ones, each from the device
    copy u0 of u^n; live kernel timing on over the timed ones.  Returns
    (wall s, per-step stats, stats after the last step)."""
    import torch
    for _ in range(warmup):
        ctx.vfs_set_velocity(u0)
        ctx.vfs_step(dt)
    ctx.vfs_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for _ in range(steps):
        ctx.vfs_set_velocity(u0)
        ctx.vfs_step(dt)
        per.append(ctx.vfs_get_stats())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ctx.vfs_get_stats()
    ctx.vfs_set_profiling(False)
    return t1 - t0, per, st


def device_faces(case, dev):
    import numpy as np
    import torch
    return [torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64).ravel(order="F"))).to(dev)
            for a in case["u"]]


def pool512_leg(V, dev, stream, steps, warmup):
    """The 2D 512^2 configuration: mixed Jacobi PCG to 1e-6, `steps` timed
    steps, with the live roofline of its dominant kernel (the fused 2D PCG
    iteration).  Returns with the figures host copies of the velocity,
    solution and active set for the CPU leg to check."""
    import cases
    case = cases.pool512()
    ctx = V.context_from_case(case, precision=V.VFS_MIXED, tol=1e-6)
    ctx.vfs_set_stream(stream.cuda_stream)
    u0 = device_faces(case, dev)
    wall, per, st = timed_steps(ctx, u0, case["dt"], steps, warmup)
    n_act = per[-1]["n_active"]
    dof_iters = sum(q["n_active"] * q["iterations"] for q in per)
    b2, t2 = fused2d_bytes(n_act), st["t_apply_avg_ms"]
    a2 = b2 / (t2 * 1e-3) / 1e9 if t2 > 0 else 0.0
    out = {"workload": "2D 512^2 pool + 8 circles + moving solid disc, mu log-uniform [1,1000] "
                       "smooth, rho [0.5,2], dt 1e-3, seed 2, mixed Jacobi PCG to 1e-6",
           "steps": steps, "warmup": warmup, "dof_iter_per_s": dof_iters / wall,
           "ms_per_step": 1e3 * wall / steps, "n_active": int(n_act),
           "cg_iterations_per_step": [q["iterations"] for q in per],
           "solve_ms_per_step": [round(q["t_solve_ms"], 3) for q in per],
           "rel_residual_fp64": [q["rel_residual"] for q in per],
           "roofline": {"bound": "hbm", "kernel": "k_fused2d (one launch per PCG iteration)",
                        "achieved": a2, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": a2 / HBM_PEAK_GBS, "traffic": measured_traffic_2d(),
                        "avg_launch_ms": t2, "launches_timed": int(st["n_apply_timed"]),
                        "algorithmic_bytes_per_launch": b2}}
    got = {"velocity": ctx.vfs_get_velocity(), "solution": ctx.vfs_get_solution(),
           "active": ctx.vfs_get_active()}
    ctx.close()
    return out, got, case


def learned_leg(V, ctx, case, u0, plain_solve_ms, plain_iters, max_iter, weights=None):
    """Flexible CG with the committed network on the headline step, to 1e-6
    or `max_iter` iterations, beside the plain Jacobi-PCG solve of the same
    step.  Non-convergence is reported as such, with the residual reached."""
    import numpy as np
    weights = weights or WEIGHTS
    w = np.load(weights, allow_pickle=False).astype(np.float32)
    ctx.vfs_load_preconditioner(w)
    ctx.vfs_set_solver(V.VFS_PRECOND_LEARNED, V.VFS_MIXED, 1e-6, max_iter)
    ctx.vfs_set_velocity(u0)
    ctx.vfs_set_profiling(True)
    ctx.vfs_step(case["dt"], allow_unconverged=True)
    sl = ctx.vfs_get_stats()
    ctx.vfs_set_profiling(False)
    ctx.vfs_set_preconditioner(None)
    ctx.vfs_set_solver(V.VFS_PRECOND_JACOBI, V.VFS_MIXED, 1e-6, 200000)
    conv = sl["rel_residual"] <= 1e-6
    return {"weights": os.path.relpath(weights, ROOT), "iteration_cap": max_iter,
            "converged": bool(conv), "iterations": sl["iterations"],
            "solve_ms": sl["t_solve_ms"], "rel_residual_fp64": sl["rel_residual"],
            "ms_per_iteration": sl["t_solve_ms"] / max(1, sl["iterations"]),
            "precond_avg_ms": sl["t_precond_avg_ms"], "fallbacks": sl["precond_fallbacks"],
            "plain_jacobi_pcg": {"iterations": plain_iters, "solve_ms": plain_solve_ms},
            "wall_time_ratio_learned_over_plain":
                (sl["t_solve_ms"] / plain_solve_ms) if conv and plain_solve_ms > 0 else None,
            "note": "learned FCG to 1e-6 against Jacobi PCG to 1e-6 on the same step"
                    if conv else f"learned FCG did not reach 1e-6 within {max_iter} iterations"}


def plain_preconditioners_leg(V, cases_list):
    """The plain preconditioners on the same FP64 steps, to 1e-6: Jacobi,
    block symmetric Gauss-Seidel on bricks (VFS_PRECOND_IC) and overlapping
    additive Schwarz on bricks (VFS_PRECOND_SCHWARZ), iterations and solve
    time per configuration (live timing of the Schwarz application)."""
    out = {}
    for label, case in cases_list:
        ctx = V.context_from_case(case, precision=V.VFS_FP64, tol=1e-6)
        res = {}
        for name, pc in (("jacobi", V.VFS_PRECOND_JACOBI), ("block_sgs", V.VFS_PRECOND_IC),
                         ("schwarz", V.VFS_PRECOND_SCHWARZ)):
            ctx.vfs_set_solver(pc, V.VFS_FP64, 1e-6, 200000)
            ctx.vfs_set_velocity(case["u"])
            ctx.vfs_set_profiling(True)
            ctx.vfs_step(case["dt"])
            st = ctx.vfs_get_stats()
            ctx.vfs_set_profiling(False)
            res[name] = {"iterations": st["iterations"], "solve_ms": st["t_solve_ms"],
                         "ms_per_iteration": st["t_solve_ms"] / max(1, st["iterations"]),
                         "rel_residual_fp64": st["rel_residual"],
                         "precond_avg_ms": st["t_precond_avg_ms"] if pc != V.VFS_PRECOND_JACOBI else None,
                         "n_active": st["n_active"]}
        ctx.close()
        out[label] = res
    return out


def hbm_copy_probe(mib=1024, reps=3, quiet=False):
    """A plain device copy of known size for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE readings into bytes: y = x + 0 over mib MiB of float32 reads
    and writes exactly mib MiB each, far more than every cache level holds.
    Returns (and unless quiet prints) the copy's own rate, read + write: what
    a plain streaming kernel reaches on this GPU, beside the 8 TB/s peak."""
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        torch.add(x, 0.0, out=y)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
    res = {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps,
           "copy_ms": ms, "copy_tb_per_s_best": 8 * n / min(ms) / 1e9}
    del x, y
    if not quiet:
        print(json.dumps(res), flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-check", action="store_true", help="skip the oracle comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--cpu-iters", type=int, default=400)
    ap.add_argument("--cpu-crop", type=int, default=64)
    ap.add_argument("--learned-max-iter", type=int, default=6000)
    ap.add_argument("--weights", default=None, help="network weights (.npy) of the learned leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-FCG leg")
    ap.add_argument("--no-pool512", action="store_true", help="skip the 2D 512^2 leg")
    ap.add_argument("--pool512-steps", type=int, default=10)
    ap.add_argument("--no-column128", action="store_true",
                    help="skip the 128^3 FP64-vs-mixed leg")
    ap.add_argument("--no-batch64", action="store_true",
                    help="skip the batched 64-problem 2D leg")
    ap.add_argument("--no-plain-precond", action="store_true",
                    help="skip the FP64 Jacobi / block-SGS / Schwarz comparison")
    ap.add_argument("--hbm-copy-probe", action="store_true",
                    help="only run the 1 GiB device copy used to scale HBM counters")
    ap.add_argument("--only", choices=["pool512", "column128", "batch64", "learned", "preconds"],
                    default=None,
                    help="run only this leg and print its figures (for profiling its kernels)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.hbm_copy_probe:
        hbm_copy_probe()
        return

    import cases
    from cases import crop_maps
    from paper_1010_2832_amd import vfstokes as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.only == "pool512":
        leg, _, _ = pool512_leg(V, dev, stream, args.pool512_steps, 2)
        print(json.dumps({"pool512_2d": leg}), flush=True)
        return
    if args.only == "column128":
        leg, _ = column128_leg(V)
        print(json.dumps({"column128_fp64_vs_mixed": leg}), flush=True)
        return
    if args.only == "batch64":
        leg, _ = batch64_leg(V)
        print(json.dumps({"batch64_2d": leg}), flush=True)
        return
    if args.only == "preconds":
        leg = plain_preconditioners_leg(V, [("pool256", cases.pool256()),
                                            ("pool512_2d", cases.pool512())])
        print(json.dumps({"plain_preconditioners_fp64": leg}), flush=True)
        return
    if args.only == "learned":
        case = cases.pool256(seed=args.seed, n=args.n)
        ctx = V.context_from_case(case, precision=V.VFS_MIXED, tol=1e-6)
        ctx.vfs_set_stream(stream.cuda_stream)
        u0 = device_faces(case, dev)
        leg = learned_leg(V, ctx, case, u0, 0.0, 0, args.learned_max_iter, args.weights)
        ctx.close()
        print(json.dumps({"learned": leg}), flush=True)
        return
    case = cases.pool256(seed=args.seed, n=args.n)
    ctx = V.context_from_case(case, precision=V.VFS_MIXED, tol=1e-6)
    ctx.vfs_set_solver(V.VFS_PRECOND_JACOBI, V.VFS_MIXED, 1e-6, 200000)
    ctx.vfs_set_stream(stream.cuda_stream)
    u0 = device_faces(case, dev)
    torch.cuda.synchronize()
    print(f"[bench] headline: {case['name']} n={args.n} seed={args.seed}", file=sys.stderr,
          flush=True)
    wall, per, st = timed_steps(ctx, u0, case["dt"], args.steps, args.warmup)
    n_act = per[-1]["n_active"]
    dof_iters = sum(q["n_active"] * q["iterations"] for q in per)
    ta = st["t_apply_avg_ms"]
    bytes_ = fused3d_bytes(n_act)
    achieved = bytes_ / (ta * 1e-3) / 1e9 if ta > 0 else 0.0
    solve_ms = [q["t_solve_ms"] for q in per]
    out = {
        "metric": "PCG solve time/step & DOF*iter/s at 1e-6 rel residual; learned vs plain PCG",
        "value": dof_iters / wall,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded generator, inputs resident in HBM)",
        "config": {"workload": f"3D {args.n}^3 pool (depth 0.3) + 8 spheres + moving solid "
                               "sphere, mu log-uniform [1,1000] smooth, rho [0.5,2], g (0,-9.8,0), "
                               "dt 1e-3, plain Jacobi PCG in mixed precision (FP32 stencil, FP64 "
                               "reductions and refinement) to 1e-6 FP64 relative residual",
                   "seed": args.seed, "n": args.n, "tol": 1e-6, "precision": "mixed",
                   "precond": "jacobi", "n_active": int(n_act),
                   "cg_iterations_per_step": [q["iterations"] for q in per],
                   "solve_ms_per_step": [round(q, 3) for q in solve_ms],
                   "rel_residual_fp64": [q["rel_residual"] for q in per],
                   "assemble_ms": st["t_assemble_ms"], "recover_ms": st["t_recover_ms"]},
        "roofline": {"bound": "hbm",
                     "kernel": "k_fused3d (one launch per PCG iteration: lazy x, r update, "
                               "Jacobi, direction, matrix-free A p, five FP64 partials)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic_3d(),
                     "avg_launch_ms": ta, "launches_timed": int(st["n_apply_timed"]),
                     "algorithmic_bytes_per_launch": bytes_,
                     "algorithmic_bytes_per_dof": bytes_ / max(n_act, 1)},
    }
    # the reachable streaming rate of this GPU, measured after the timed steps
    cp = hbm_copy_probe(reps=4, quiet=True)
    out["hbm_copy"] = {"tb_per_s": cp["copy_tb_per_s_best"],
                       "bytes_per_copy": cp["copy_bytes_read"] + cp["copy_bytes_written"],
                       "note": "plain 1 GiB device copy (read + write), best of 4; the fused "
                               "kernel's measured traffic rate is traffic / avg_launch_ms"}
    out["paper_context"] = {
        "timings": None,
        "note": "the paper reports no wall-clock times, hardware or precision; its only solver "
                "figures are PCG iteration counts with an overlapping multiplicative Schwarz "
                "preconditioner (Table 1, 2D only), against Jacobi PCG here"}
    head_got = {"velocity": ctx.vfs_get_velocity(), "solution": ctx.vfs_get_solution(),
                "rhs": ctx.vfs_get_rhs(), "active": ctx.vfs_get_active()}
    if not args.no_learned and os.path.exists(WEIGHTS):
        print("[bench] learned FCG leg", file=sys.stderr, flush=True)
        plain_ms = sorted(solve_ms)[len(solve_ms) // 2]
        out["learned_vs_plain"] = learned_leg(V, ctx, case, u0, plain_ms,
                                              per[-1]["iterations"], args.learned_max_iter,
                                              args.weights)
    ctx.close()
    extra3d = [("headline", case, crop_maps.sites_pool, {"plain_jacobi_pcg": head_got})]
    extra2d, batch_got = [], None
    if not args.no_pool512:
        print("[bench] 512^2 leg", file=sys.stderr, flush=True)
        out["pool512_2d"], got2, c2 = pool512_leg(V, dev, stream, args.pool512_steps, 2)
        extra2d.append(("pool512_2d", c2, got2))
    if not args.no_column128:
        print("[bench] 128^3 column leg", file=sys.stderr, flush=True)
        out["column128_fp64_vs_mixed"], got = column128_leg(V)
        extra3d.append(("column128_fp64_vs_mixed", cases.column128(), crop_maps.sites_column, got))
    if not args.no_batch64:
        print("[bench] batched 2D leg", file=sys.stderr, flush=True)
        out["batch64_2d"], batch_got = batch64_leg(V)
    if not args.no_plain_precond:
        print("[bench] plain preconditioners leg", file=sys.stderr, flush=True)
        out["plain_preconditioners_fp64"] = plain_preconditioners_leg(
            V, [("pool256", cases.pool256()), ("pool512_2d", cases.pool512())])
    base_case = None
    if not args.no_cpu:
        lo = crop_maps.crop_lo(case, (0.5, 0.3, 0.5), args.cpu_crop)
        base_case = cases.crop(case, lo, (args.cpu_crop,) * 3)
    del u0, head_got
    if not (args.no_check and args.no_cpu):
        print("[bench] CPU oracle leg", file=sys.stderr, flush=True)
        res = cpu_oracle_leg(base_case, args.cpu_iters, None, batch_got,
                             baseline=not args.no_cpu, check=not args.no_check,
                             extra3d=extra3d, extra2d=extra2d)
        if "cpu_baseline" in res:
            out["cpu_baseline"] = res["cpu_baseline"]
        if "headline" in res:
            out["error_vs_fp64_oracle"] = res["headline"]
        if "batch64_error_vs_fp64_oracle" in res:
            out["batch64_2d"]["error_vs_fp64_oracle"] = res["batch64_error_vs_fp64_oracle"]
        for key, _, _, _ in extra3d[1:]:
            if key in res:
                out[key]["error_vs_fp64_oracle"] = res[key]
        for key, _, _ in extra2d:
            if key in res:
                out[key]["error_vs_fp64_oracle"] = res[key]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
