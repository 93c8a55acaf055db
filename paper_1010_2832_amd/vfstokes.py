"""Thin ctypes binding of libvfstokes.so (the C ABI declared in
include/vfstokes.h).  Functions keep the C names; this module only
marshals arguments: NumPy arrays indexed [i, j(, k)] are flattened x-fastest,
torch tensors (host or device, float64, contiguous, already x-fastest) are
passed by pointer so that data resident in HBM is never copied through the
host.  Every numerical step runs inside the HIP library; if the library is
missing this module raises at import time.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvfstokes.so")

VFS_OK, VFS_EINVAL, VFS_ENOMEM, VFS_EHIP, VFS_ENOTCONV, VFS_EBREAKDOWN, VFS_ESTATE = 0, -1, -2, -3, -4, -5, -6
VFS_PRECOND_NONE, VFS_PRECOND_JACOBI, VFS_PRECOND_IC, VFS_PRECOND_LEARNED = 0, 1, 2, 3
VFS_PRECOND_SCHWARZ = 4
VFS_SAMPLE_P, VFS_SAMPLE_TXX = 0, 1
VFS_SAMPLE_TXY_2D = 2
VFS_SAMPLE_TYY, VFS_SAMPLE_TXY, VFS_SAMPLE_TXZ, VFS_SAMPLE_TYZ = 2, 3, 4, 5
VFS_FP64, VFS_MIXED = 0, 1
VFS_SET_CELL, VFS_SET_FACE_X, VFS_SET_FACE_Y, VFS_SET_FACE_Z = 0, 1, 2, 3
VFS_SET_NODE = VFS_SET_EDGE_Z = 4
VFS_SET_EDGE_Y, VFS_SET_EDGE_X = 5, 6
VFS_WEIGHT_LIQUID, VFS_WEIGHT_FLUID = 0, 1

_CODES = {0: "VFS_OK", -1: "VFS_EINVAL", -2: "VFS_ENOMEM", -3: "VFS_EHIP", -4: "VFS_ENOTCONV",
          -5: "VFS_EBREAKDOWN", -6: "VFS_ESTATE"}


class vfs_stats(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_active", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("outer_iterations", ctypes.c_int32),
                ("status", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("b_norm", ctypes.c_double),
                ("t_assemble_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("t_recover_ms", ctypes.c_double), ("t_step_ms", ctypes.c_double),
                ("t_apply_avg_ms", ctypes.c_double), ("t_update_avg_ms", ctypes.c_double),
                ("n_apply_timed", ctypes.c_int64), ("n_update_timed", ctypes.c_int64),
                ("t_precond_avg_ms", ctypes.c_double), ("precond_fallbacks", ctypes.c_int32),
                ("pad0", ctypes.c_int32), ("n_tile_samples", ctypes.c_int64),
                ("rel_residual_start", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}


class vfs_batch_stats(ctypes.Structure):
    _fields_ = [("n_problems", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("graph_used", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_active_total", ctypes.c_int64), ("dof_iters", ctypes.c_int64),
                ("max_iterations", ctypes.c_int32), ("passes_max", ctypes.c_int32),
                ("t_assemble_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("t_step_ms", ctypes.c_double), ("latency_p50_ms", ctypes.c_double),
                ("latency_p90_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("n_items", ctypes.c_int64),
                ("n_tile_samples", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class VfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


def _load():
    # torch ships its own HIP runtime with the same soname as the system one.
    # Loading torch first makes this library bind to that runtime, so the
    # process has one HIP runtime and torch streams / device pointers are
    # valid handles for the library.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run paper_1010_2832_amd/build.py)")
    return ctypes.CDLL(LIB_PATH)


_lib = _load()
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_SIGS = {
    "vfs_last_error": ([_P], ctypes.c_char_p),
    "vfs_create": ([ctypes.POINTER(_P), _I, _I, _I, _I, _D, _P], _I),
    "vfs_destroy": ([_P], _I),
    "vfs_set_stream": ([_P, _P], _I),
    "vfs_set_level_sets": ([_P, _P, _P], _I),
    "vfs_set_density": ([_P, _P], _I),
    "vfs_set_viscosity": ([_P, _P], _I),
    "vfs_set_velocity": ([_P, _P, _P, _P], _I),
    "vfs_set_solid_velocity": ([_P, _P, _P, _P], _I),
    "vfs_set_gravity": ([_P, _P], _I),
    "vfs_set_traction": ([_P, _P, _P], _I),
    "vfs_advect": ([_P, _D], _I),
    "vfs_get_level_set": ([_P, _P], _I),
    "vfs_set_warm_start": ([_P, _I], _I),
    "vfs_set_solver": ([_P, _I, _I, _D, _I, _D], _I),
    "vfs_step": ([_P, _D], _I),
    "vfs_assemble": ([_P, _D], _I),
    "vfs_apply": ([_P, _P, _P], _I),
    "vfs_solve": ([_P, _P, _P], _I),
    "vfs_get_velocity": ([_P, _P, _P, _P], _I),
    "vfs_get_pressure": ([_P, _P], _I),
    "vfs_get_stress": ([_P, _P], _I),
    "vfs_get_solution": ([_P, _P], _I),
    "vfs_get_rhs": ([_P, _P], _I),
    "vfs_get_weights": ([_P, _I, _I, _P], _I),
    "vfs_get_active": ([_P, _P], _I),
    "vfs_get_active_mask": ([_P, _I, _P], _I),
    "vfs_training_pair": ([_P, _P, _P, _P, _P], _I),
    "vfs_get_stats": ([_P, ctypes.POINTER(vfs_stats)], _I),
    "vfs_get_sizes": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], _I),
    "vfs_set_profiling": ([_P, _I], _I),
    "vfs_batch_last_error": ([_P], ctypes.c_char_p),
    "vfs_batch_create": ([ctypes.POINTER(_P), _I, _P, _P, _P], _I),
    "vfs_batch_destroy": ([_P], _I),
    "vfs_batch_set_stream": ([_P, _P], _I),
    "vfs_batch_set_problem": ([_P, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I),
    "vfs_batch_set_solver": ([_P, _D, _I, _D], _I),
    "vfs_batch_num_variants": ([], _I),
    "vfs_batch_variant_shape": ([_I, ctypes.POINTER(_I), ctypes.POINTER(_I)], _I),
    "vfs_batch_max_blocks_per_cu": ([_I], _I),
    "vfs_batch_set_tiles": ([_P, _I, _I], _I),
    "vfs_batch_time_variant": ([_P, _I, _I, _I, ctypes.POINTER(_D)], _I),
    "vfs_batch_step": ([_P, _D], _I),
    "vfs_batch_get_velocity": ([_P, _I, _P, _P], _I),
    "vfs_batch_get_solution": ([_P, _I, _P], _I),
    "vfs_batch_get_problem": ([_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_D),
                               ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_int64)], _I),
    "vfs_batch_get_stats": ([_P, ctypes.POINTER(vfs_batch_stats)], _I),
    "vfs_unet_last_error": ([_P], ctypes.c_char_p),
    "vfs_unet_param_count": ([], ctypes.c_int64),
    "vfs_unet_create": ([ctypes.POINTER(_P)], _I),
    "vfs_unet_destroy": ([_P], _I),
    "vfs_unet_set_stream": ([_P, _P], _I),
    "vfs_unet_set_weights": ([_P, _P, ctypes.c_int64], _I),
    "vfs_unet_get_weights": ([_P, _P, ctypes.c_int64], _I),
    "vfs_unet_get_grad": ([_P, _P, ctypes.c_int64], _I),
    "vfs_unet_zero_grad": ([_P], _I),
    "vfs_unet_forward": ([_P, _I, _I, _I, _P, _P], _I),
    "vfs_unet_backward": ([_P, _P], _I),
    "vfs_unet_adam": ([_P, _D, _D, _D, _D, _D], _I),
    "vfs_unet_train_step": ([_P, _P, _P, _P, ctypes.POINTER(_D)], _I),
    "vfs_set_preconditioner": ([_P, _P], _I),
    "vfs_load_preconditioner": ([_P, _P, ctypes.c_size_t], _I),
    "vfs_liquid_weights_noalloc": ([_I, _I, _I, _I, _D, _P, _I, _P, _P], _I),
    "vfs_precond_apply": ([_P, _P, _P], _I),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


# ---------------------------------------------------------------------------
# shapes
# ---------------------------------------------------------------------------
def set_shape(dim, n, s):
    """Native shape of a sample set (stagger s per axis: 1 cell-centred)."""
    return tuple(n[a] + 1 - s[a] for a in range(dim))


def sample_staggers(dim):
    if dim == 2:
        return [(1, 1), (1, 1), (0, 0)]
    return [(1, 1, 1)] * 3 + [(0, 0, 1), (0, 1, 0), (1, 0, 0)]


def face_staggers(dim):
    return [tuple(0 if b == a else 1 for b in range(dim)) for a in range(dim)]


# ---------------------------------------------------------------------------
# marshalling
# ---------------------------------------------------------------------------
def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Keep:
    """Holds converted buffers alive for the duration of one call."""

    def __init__(self):
        self.items = []

    def ptr(self, arr, n=None):
        if arr is None:
            return None
        if _is_torch(arr):
            import torch
            if arr.dtype != torch.float64 or not arr.is_contiguous():
                raise ValueError("torch tensors must be contiguous float64")
            if n is not None and arr.numel() != n:
                raise ValueError(f"expected {n} values, got {arr.numel()}")
            return arr.data_ptr()
        flat = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).ravel(order="F"))
        if n is not None and flat.size != n:
            raise ValueError(f"expected {n} values, got {flat.size}")
        self.items.append(flat)
        return flat.ctypes.data


def _ptr32(keep, arr, n):
    """float32 buffer pointer: torch float32 tensors by pointer, anything
    else converted to a contiguous float32 NumPy array (C order)."""
    if _is_torch(arr):
        import torch
        if arr.dtype != torch.float32 or not arr.is_contiguous():
            raise ValueError("torch tensors must be contiguous float32")
        if arr.numel() != n:
            raise ValueError(f"expected {n} values, got {arr.numel()}")
        return arr.data_ptr()
    flat = np.ascontiguousarray(np.asarray(arr, dtype=np.float32).ravel())
    if flat.size != n:
        raise ValueError(f"expected {n} values, got {flat.size}")
    keep.items.append(flat)
    return flat.ctypes.data


def _check(ctx, rc, allow=(VFS_OK,)):
    if rc not in allow:
        raise VfsError(rc, _lib.vfs_last_error(ctx).decode())
    return rc


# ---------------------------------------------------------------------------
# same-name wrappers
# ---------------------------------------------------------------------------
def vfs_create(dim, nx, ny, nz, h, origin=None):
    out = _P()
    org = (ctypes.c_double * 3)(*((list(origin) + [0.0] * 3)[:3] if origin is not None else [0.0] * 3))
    rc = _lib.vfs_create(ctypes.byref(out), dim, nx, ny, nz, h, ctypes.cast(org, _P))
    if rc != VFS_OK:
        raise VfsError(rc, _lib.vfs_last_error(None).decode())
    return out


def vfs_destroy(ctx):
    return _lib.vfs_destroy(ctx)


def vfs_liquid_weights_noalloc(dim, n, w_min, phi_liquid, set_id, out, stream_ptr=None):
    """W_L of one sample set from a nodal liquid level set, allocating nothing.
    phi_liquid and out are contiguous torch float64 tensors on the GPU (the
    level set flattened x-fastest, out sized for the set); work is queued on
    stream_ptr and not synchronised."""
    nx, ny = int(n[0]), int(n[1])
    nz = int(n[2]) if dim == 3 else 1
    for t in (phi_liquid, out):
        if not _is_torch(t) or not t.is_cuda or not t.is_contiguous():
            raise ValueError("phi_liquid and out must be contiguous torch tensors on the GPU")
    rc = _lib.vfs_liquid_weights_noalloc(dim, nx, ny, nz, float(w_min), phi_liquid.data_ptr(),
                                         int(set_id), out.data_ptr(), stream_ptr)
    if rc != VFS_OK:
        raise VfsError(rc, _lib.vfs_last_error(None).decode())
    return rc


def vfs_set_stream(ctx, stream_ptr):
    return _check(ctx, _lib.vfs_set_stream(ctx, stream_ptr))


class Context:
    """Owns one vfs_ctx.  Method names follow the C entry points."""

    def __init__(self, dim, n, h, origin=None):
        self.dim = int(dim)
        self.n = tuple(int(q) for q in n)
        nz = self.n[2] if self.dim == 3 else 1
        self.h = float(h)
        self.handle = vfs_create(self.dim, self.n[0], self.n[1], nz, self.h, origin)

    def close(self):
        if self.handle:
            _lib.vfs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # sizes -----------------------------------------------------------------
    def node_shape(self):
        return tuple(q + 1 for q in self.n)

    def cell_shape(self):
        return self.n

    def face_shapes(self):
        return [set_shape(self.dim, self.n, s) for s in face_staggers(self.dim)]

    def sample_shapes(self):
        return [set_shape(self.dim, self.n, s) for s in sample_staggers(self.dim)]

    def n_samples(self):
        return int(sum(np.prod(s) for s in self.sample_shapes()))

    # inputs ----------------------------------------------------------------
    def vfs_set_stream(self, stream_ptr):
        return _check(self.handle, _lib.vfs_set_stream(self.handle, stream_ptr))

    def vfs_set_level_sets(self, phi_l, phi_s=None):
        k = _Keep()
        nn = int(np.prod(self.node_shape()))
        return _check(self.handle, _lib.vfs_set_level_sets(self.handle, k.ptr(phi_l, nn), k.ptr(phi_s, nn)))

    def vfs_set_density(self, rho):
        k = _Keep()
        return _check(self.handle, _lib.vfs_set_density(self.handle, k.ptr(rho, int(np.prod(self.n)))))

    def vfs_set_viscosity(self, mu):
        k = _Keep()
        return _check(self.handle, _lib.vfs_set_viscosity(self.handle, k.ptr(mu, int(np.prod(self.n)))))

    def _faces(self, comps):
        k = _Keep()
        fs = self.face_shapes()
        ptrs = [None, None, None]
        if comps is not None:
            for a in range(self.dim):
                ptrs[a] = k.ptr(comps[a], int(np.prod(fs[a])))
        return k, ptrs

    def vfs_set_velocity(self, u):
        k, p = self._faces(u)
        return _check(self.handle, _lib.vfs_set_velocity(self.handle, *p))

    def vfs_set_solid_velocity(self, ubc=None):
        k, p = self._faces(ubc)
        return _check(self.handle, _lib.vfs_set_solid_velocity(self.handle, *p))

    def vfs_set_gravity(self, g):
        arr = (ctypes.c_double * 3)(*((list(g) + [0.0] * 3)[:3]))
        return _check(self.handle, _lib.vfs_set_gravity(self.handle, ctypes.cast(arr, _P)))

    def vfs_set_traction(self, p_bc=None, tau_bc=None):
        """Prescribed pressure (cells) and deviatoric stresses (list in sample
        order after p, native shapes; None entries mean 0)."""
        k = _Keep()
        shapes = self.sample_shapes()
        pp = k.ptr(p_bc, int(np.prod(shapes[0]))) if p_bc is not None else None
        arr = None
        if tau_bc is not None:
            ptrs = [k.ptr(t, int(np.prod(shapes[q + 1]))) if t is not None else None
                    for q, t in enumerate(tau_bc)]
            arr = (_P * len(ptrs))(*ptrs)
        return _check(self.handle, _lib.vfs_set_traction(self.handle, pp,
                                                         ctypes.cast(arr, _P) if arr is not None else None))

    def vfs_advect(self, dt):
        return _check(self.handle, _lib.vfs_advect(self.handle, dt))

    def vfs_get_level_set(self):
        out = np.zeros(int(np.prod([q + 1 for q in self.n])))
        _check(self.handle, _lib.vfs_get_level_set(self.handle, out.ctypes.data))
        return out.reshape(tuple(q + 1 for q in self.n), order="F")

    def vfs_set_warm_start(self, on=True):
        return _check(self.handle, _lib.vfs_set_warm_start(self.handle, 1 if on else 0))

    def vfs_set_solver(self, precond=VFS_PRECOND_JACOBI, precision=VFS_FP64, rel_tol=1e-6,
                       max_iter=100000, w_min=1e-3):
        rc = _check(self.handle, _lib.vfs_set_solver(self.handle, precond, precision, rel_tol,
                                                     max_iter, w_min))
        self._solver = (precond, precision, rel_tol, max_iter, w_min)
        return rc

    # work ------------------------------------------------------------------
    def vfs_step(self, dt, allow_unconverged=False):
        allow = (VFS_OK, VFS_ENOTCONV, VFS_EBREAKDOWN) if allow_unconverged else (VFS_OK,)
        return _check(self.handle, _lib.vfs_step(self.handle, dt), allow)

    def vfs_assemble(self, dt):
        return _check(self.handle, _lib.vfs_assemble(self.handle, dt))

    def vfs_apply(self, x):
        k = _Keep()
        n = self.n_samples()
        y = np.zeros(n)
        _check(self.handle, _lib.vfs_apply(self.handle, k.ptr(x, n), y.ctypes.data))
        return y

    def vfs_solve(self, b, allow_unconverged=False):
        k = _Keep()
        n = self.n_samples()
        x = np.zeros(n)
        allow = (VFS_OK, VFS_ENOTCONV, VFS_EBREAKDOWN) if allow_unconverged else (VFS_OK,)
        _check(self.handle, _lib.vfs_solve(self.handle, k.ptr(b, n), x.ctypes.data), allow)
        return x

    # outputs ---------------------------------------------------------------
    def vfs_get_velocity(self):
        fs = self.face_shapes()
        outs = [np.zeros(int(np.prod(s))) for s in fs] + [None] * (3 - self.dim)
        ptrs = [o.ctypes.data if o is not None else None for o in outs]
        _check(self.handle, _lib.vfs_get_velocity(self.handle, *ptrs))
        return [outs[a].reshape(fs[a], order="F") for a in range(self.dim)]

    def vfs_get_pressure(self):
        p = np.zeros(int(np.prod(self.n)))
        _check(self.handle, _lib.vfs_get_pressure(self.handle, p.ctypes.data))
        return p.reshape(self.n, order="F")

    def vfs_get_stress(self):
        shapes = self.sample_shapes()[1:]
        outs = [np.zeros(int(np.prod(s))) for s in shapes]
        arr = (_P * len(outs))(*[o.ctypes.data for o in outs])
        _check(self.handle, _lib.vfs_get_stress(self.handle, ctypes.cast(arr, _P)))
        return [o.reshape(s, order="F") for o, s in zip(outs, shapes)]

    def vfs_get_solution(self):
        x = np.zeros(self.n_samples())
        _check(self.handle, _lib.vfs_get_solution(self.handle, x.ctypes.data))
        return x

    def vfs_get_rhs(self):
        b = np.zeros(self.n_samples())
        _check(self.handle, _lib.vfs_get_rhs(self.handle, b.ctypes.data))
        return b

    def vfs_get_weights(self, set_id, which):
        if self.dim == 2:
            st = {VFS_SET_CELL: (1, 1), VFS_SET_FACE_X: (0, 1), VFS_SET_FACE_Y: (1, 0), VFS_SET_NODE: (0, 0)}[set_id]
        else:
            st = [(1, 1, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)][set_id]
        shp = set_shape(self.dim, self.n, st)
        out = np.zeros(int(np.prod(shp)))
        _check(self.handle, _lib.vfs_get_weights(self.handle, set_id, which, out.ctypes.data))
        return out.reshape(shp, order="F")

    def vfs_get_active(self):
        out = np.zeros(self.n_samples(), dtype=np.uint8)
        _check(self.handle, _lib.vfs_get_active(self.handle, out.ctypes.data))
        return out.astype(bool)

    def vfs_get_active_mask(self, sample):
        shp = self.sample_shapes()[sample] if 0 <= sample < len(self.sample_shapes()) else (0,)
        out = np.zeros(int(np.prod(shp)), dtype=np.uint8)
        _check(self.handle, _lib.vfs_get_active_mask(self.handle, sample, out.ctypes.data))
        return out.reshape(shp, order="F").astype(bool)

    def vfs_training_pair(self, x_star, x_k):
        k = _Keep()
        n = self.n_samples()
        r = np.zeros(n)
        e = np.zeros(n)
        _check(self.handle, _lib.vfs_training_pair(self.handle, k.ptr(x_star, n), k.ptr(x_k, n),
                                                   r.ctypes.data, e.ctypes.data))
        return r, e

    def vfs_get_stats(self):
        st = vfs_stats()
        _check(self.handle, _lib.vfs_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def vfs_set_profiling(self, on=True):
        return _check(self.handle, _lib.vfs_set_profiling(self.handle, 1 if on else 0))

    def vfs_get_sizes(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(self.handle, _lib.vfs_get_sizes(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # learned preconditioner -------------------------------------------------
    def vfs_set_preconditioner(self, net):
        self._net = net   # the context does not own the network; keep it alive
        return _check(self.handle, _lib.vfs_set_preconditioner(self.handle,
                                                               net.handle if net else None))

    def vfs_load_preconditioner(self, weights):
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
        self._net = None   # the context owns the network it loads
        return _check(self.handle, _lib.vfs_load_preconditioner(self.handle, w.ctypes.data,
                                                                w.nbytes))

    def vfs_precond_apply(self, r):
        k = _Keep()
        n = self.n_samples()
        z = np.zeros(n)
        _check(self.handle, _lib.vfs_precond_apply(self.handle, k.ptr(r, n), z.ctypes.data))
        return z


def context_from_case(case, precision=VFS_FP64, tol=None, max_iter=200000, w_min=1e-3):
    """Create a context and load a case dict (the format of the ``cases``
    generators) into it."""
    ctx = Context(case["dim"], case["n"], case["h"], case.get("origin"))
    ctx.vfs_set_level_sets(case["phi_l"], case.get("phi_s"))
    ctx.vfs_set_density(case["rho"])
    ctx.vfs_set_viscosity(case["mu"])
    ctx.vfs_set_velocity(case["u"])
    ctx.vfs_set_solid_velocity(case.get("u_bc"))
    ctx.vfs_set_gravity(case["g"])
    if case.get("p_bc") is not None or case.get("tau_bc") is not None:
        ctx.vfs_set_traction(case.get("p_bc"), case.get("tau_bc"))
    ctx.vfs_set_solver(VFS_PRECOND_JACOBI, precision, tol if tol is not None else case.get("tol", 1e-6),
                       max_iter, w_min)
    return ctx


# ---------------------------------------------------------------------------
# batched 2D steps
# ---------------------------------------------------------------------------
def _bcheck(b, rc, allow=(VFS_OK,)):
    if rc not in allow:
        raise VfsError(rc, _lib.vfs_batch_last_error(b).decode())
    return rc


def vfs_batch_num_variants():
    return _lib.vfs_batch_num_variants()


def vfs_batch_variant_shape(variant):
    bx, by = _I(), _I()
    _bcheck(None, _lib.vfs_batch_variant_shape(variant, ctypes.byref(bx), ctypes.byref(by)))
    return bx.value, by.value


def vfs_batch_max_blocks_per_cu(variant):
    rc = _lib.vfs_batch_max_blocks_per_cu(variant)
    if rc < 0:
        raise VfsError(rc, f"vfs_batch_max_blocks_per_cu({variant}) failed")
    return rc


class Batch:
    """Owns one vfs_batch: n independent 2D problems (sizes n_i x m_i)."""

    def __init__(self, sizes, hs):
        self.sizes = [tuple(int(q) for q in s) for s in sizes]
        n = len(self.sizes)
        nx = (ctypes.c_int * n)(*[s[0] for s in self.sizes])
        ny = (ctypes.c_int * n)(*[s[1] for s in self.sizes])
        h = (ctypes.c_double * n)(*[float(q) for q in hs])
        out = _P()
        rc = _lib.vfs_batch_create(ctypes.byref(out), n, ctypes.cast(nx, _P), ctypes.cast(ny, _P),
                                   ctypes.cast(h, _P))
        if rc != VFS_OK:
            raise VfsError(rc, _lib.vfs_batch_last_error(None).decode())
        self.handle = out
        self.n = n

    def close(self):
        if self.handle:
            _lib.vfs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vfs_batch_set_stream(self, stream_ptr):
        return _bcheck(self.handle, _lib.vfs_batch_set_stream(self.handle, stream_ptr))

    def vfs_batch_set_problem(self, i, case):
        k = _Keep()
        nx, ny = self.sizes[i]
        nn = (nx + 1) * (ny + 1)
        fs = [(nx + 1) * ny, nx * (ny + 1)]
        ubc = case.get("u_bc")
        g = (ctypes.c_double * 3)(*((list(case["g"]) + [0.0] * 3)[:3]))
        return _bcheck(self.handle, _lib.vfs_batch_set_problem(
            self.handle, i, k.ptr(case["phi_l"], nn), k.ptr(case.get("phi_s"), nn),
            k.ptr(case["rho"], nx * ny), k.ptr(case["mu"], nx * ny),
            k.ptr(case["u"][0], fs[0]), k.ptr(case["u"][1], fs[1]),
            k.ptr(ubc[0], fs[0]) if ubc is not None else None,
            k.ptr(ubc[1], fs[1]) if ubc is not None else None, ctypes.cast(g, _P)))

    def vfs_batch_set_solver(self, rel_tol=1e-6, max_iter=200000, w_min=1e-3):
        return _bcheck(self.handle, _lib.vfs_batch_set_solver(self.handle, rel_tol, max_iter, w_min))

    def vfs_batch_set_tiles(self, variant, blocks_per_cu):
        return _bcheck(self.handle, _lib.vfs_batch_set_tiles(self.handle, variant, blocks_per_cu))

    def vfs_batch_time_variant(self, variant, blocks_per_cu, iterations=50):
        ms = _D()
        _bcheck(self.handle, _lib.vfs_batch_time_variant(self.handle, variant, blocks_per_cu,
                                                         iterations, ctypes.byref(ms)))
        return ms.value

    def vfs_batch_step(self, dt, allow_unconverged=False):
        allow = (VFS_OK, VFS_ENOTCONV) if allow_unconverged else (VFS_OK,)
        return _bcheck(self.handle, _lib.vfs_batch_step(self.handle, dt), allow)

    def vfs_batch_get_velocity(self, i):
        nx, ny = self.sizes[i]
        u = np.zeros((nx + 1) * ny)
        v = np.zeros(nx * (ny + 1))
        _bcheck(self.handle, _lib.vfs_batch_get_velocity(self.handle, i, u.ctypes.data, v.ctypes.data))
        return [u.reshape((nx + 1, ny), order="F"), v.reshape((nx, ny + 1), order="F")]

    def vfs_batch_get_solution(self, i):
        nx, ny = self.sizes[i]
        x = np.zeros(2 * nx * ny + (nx + 1) * (ny + 1))
        _bcheck(self.handle, _lib.vfs_batch_get_solution(self.handle, i, x.ctypes.data))
        return x

    def vfs_batch_get_problem(self, i):
        it, ps = _I(), _I()
        rel, lat = _D(), _D()
        na = ctypes.c_int64()
        _bcheck(self.handle, _lib.vfs_batch_get_problem(self.handle, i, ctypes.byref(it), ctypes.byref(ps),
                                                        ctypes.byref(rel), ctypes.byref(lat),
                                                        ctypes.byref(na)))
        return dict(iterations=it.value, passes=ps.value, rel_residual=rel.value,
                    latency_ms=lat.value, n_active=na.value)

    def vfs_batch_get_stats(self):
        st = vfs_batch_stats()
        _bcheck(self.handle, _lib.vfs_batch_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()


def batch_from_cases(case_list, tol=1e-6, max_iter=200000, w_min=1e-3):
    b = Batch([c["n"] for c in case_list], [c["h"] for c in case_list])
    for i, c in enumerate(case_list):
        b.vfs_batch_set_problem(i, c)
    b.vfs_batch_set_solver(tol, max_iter, w_min)
    return b


# ---------------------------------------------------------------------------
# learned preconditioner network
# ---------------------------------------------------------------------------
def vfs_unet_param_count():
    return int(_lib.vfs_unet_param_count())


def _ucheck(u, rc, allow=(VFS_OK,)):
    if rc not in allow:
        raise VfsError(rc, _lib.vfs_unet_last_error(u).decode())
    return rc


class Unet:
    """Owns one vfs_unet (weights, Adam state, activation tensors)."""

    def __init__(self):
        out = _P()
        rc = _lib.vfs_unet_create(ctypes.byref(out))
        if rc != VFS_OK:
            raise VfsError(rc, _lib.vfs_unet_last_error(None).decode())
        self.handle = out
        self.n_params = vfs_unet_param_count()

    def close(self):
        if self.handle:
            _lib.vfs_unet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vfs_unet_set_stream(self, stream_ptr):
        return _ucheck(self.handle, _lib.vfs_unet_set_stream(self.handle, stream_ptr))

    def vfs_unet_set_weights(self, w):
        k = _Keep()
        return _ucheck(self.handle, _lib.vfs_unet_set_weights(
            self.handle, _ptr32(k, w, self.n_params), self.n_params))

    def vfs_unet_get_weights(self):
        w = np.zeros(self.n_params, dtype=np.float32)
        _ucheck(self.handle, _lib.vfs_unet_get_weights(self.handle, w.ctypes.data, self.n_params))
        return w

    def vfs_unet_get_grad(self):
        g = np.zeros(self.n_params, dtype=np.float32)
        _ucheck(self.handle, _lib.vfs_unet_get_grad(self.handle, g.ctypes.data, self.n_params))
        return g

    def vfs_unet_zero_grad(self):
        return _ucheck(self.handle, _lib.vfs_unet_zero_grad(self.handle))

    def vfs_unet_forward(self, x):
        """x: (Z, Y, X, 16) float array; returns y (Z, Y, X, 6) float32."""
        Z, Y, X = (int(q) for q in np.shape(x)[:3])
        k = _Keep()
        y = np.zeros((Z, Y, X, 6), dtype=np.float32)
        _ucheck(self.handle, _lib.vfs_unet_forward(self.handle, X, Y, Z,
                                                   _ptr32(k, x, Z * Y * X * 16), y.ctypes.data))
        return y

    def vfs_unet_backward(self, gy):
        Z, Y, X = (int(q) for q in np.shape(gy)[:3])
        k = _Keep()
        return _ucheck(self.handle, _lib.vfs_unet_backward(self.handle,
                                                           _ptr32(k, gy, Z * Y * X * 6)))

    def vfs_unet_adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        return _ucheck(self.handle, _lib.vfs_unet_adam(self.handle, lr, beta1, beta2, eps,
                                                       grad_scale))

    def vfs_unet_train_step(self, ctx, r, e):
        k = _Keep()
        n = ctx.n_samples()
        loss = _D()
        _ucheck(self.handle, _lib.vfs_unet_train_step(self.handle, ctx.handle, k.ptr(r, n),
                                                      k.ptr(e, n), ctypes.byref(loss)))
        return loss.value
