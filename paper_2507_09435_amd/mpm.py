"""Thin Python binding of the C ABI in include/mpm.h (argument marshalling only).

Every step of the hot path runs in the HIP library; this module only turns
torch device tensors into pointers and ctypes structs.  It raises if the
library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmpm_hip.so")

MPM_OK, MPM_E_INVALID, MPM_E_NOMEM, MPM_E_HIP = 0, -1, -2, -3
MPM_E_NOT_CONVERGED, MPM_E_KRYLOV, MPM_E_NONFINITE, MPM_E_OUT_OF_GRID, MPM_E_RANGE = -4, -5, -6, -7, -8
MPM_JAC_RAW = 1
MPM_MAX_REPORT = 32

STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "NOT_CONVERGED", -5: "KRYLOV",
                -6: "NONFINITE", -7: "OUT_OF_GRID", -8: "RANGE"}


class MPMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class mpm_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("ncell", C.c_int32 * 3), ("h", C.c_double), ("origin", C.c_double * 3)]


class mpm_material(C.Structure):
    _fields_ = [("up", C.c_int32), ("dp", C.c_int32), ("dp_match", C.c_int32), ("shape", C.c_int32),
                ("E", C.c_double), ("nu", C.c_double), ("phi", C.c_double), ("c", C.c_double), ("psi", C.c_double),
                ("rho0", C.c_double), ("g", C.c_double * 3), ("perm", C.c_double), ("mu_f", C.c_double),
                ("biot", C.c_double), ("rho_f", C.c_double), ("dt", C.c_double), ("apex_reg", C.c_double),
                ("lp0", C.c_double * 3), ("elastic", C.c_int32), ("reserved", C.c_int32)]


class mpm_particles(C.Structure):
    _fields_ = [("np", C.c_int64), ("x", C.c_void_p), ("vol0", C.c_void_p), ("F", C.c_void_p), ("be", C.c_void_p),
                ("fp", C.c_void_p), ("E", C.c_void_p), ("phi", C.c_void_p)]


class mpm_problem(C.Structure):
    _fields_ = [("nsim", C.c_int32), ("reserved", C.c_int32), ("grids", C.POINTER(mpm_grid)),
                ("sim_start", C.POINTER(C.c_int64)), ("mat", mpm_material), ("P", mpm_particles),
                ("bc_mask", C.c_void_p), ("bc_value", C.c_void_p), ("react_mask", C.c_void_p)]


class mpm_newton_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("commit", C.c_int32), ("stall_factor", C.c_double),
                ("krylov_rtol", C.c_double), ("krylov_max_iter", C.c_int32), ("line_search", C.c_int32),
                ("time_spmv", C.c_int32), ("krylov_method", C.c_int32)]


class mpm_newton_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("krylov_iters", C.c_int64),
                ("norms", C.c_double * MPM_MAX_REPORT), ("krylov", C.c_int32 * MPM_MAX_REPORT),
                ("ms_residual", C.c_double), ("ms_jacobian", C.c_double), ("ms_krylov", C.c_double),
                ("ms_total", C.c_double), ("spmv_ms", C.c_double), ("spmv_launches", C.c_int64),
                ("sim_iters", C.POINTER(C.c_int32)),
                ("sim_converged", C.POINTER(C.c_int32)), ("sim_reaction", C.POINTER(C.c_double)),
                ("sim_rel", C.POINTER(C.c_double)), ("precond_flags", C.c_int32), ("reserved", C.c_int32)]


EXPORTS = ["mpm_create", "mpm_destroy", "mpm_last_error", "mpm_prepare", "mpm_residual", "mpm_jacobian_bsr",
           "mpm_newton_step", "mpm_update", "mpm_spmv", "mpm_spmv_lanes", "mpm_spmv_set_lanes",
           "mpm_adjoint_step", "mpm_residual_noalloc", "mpm_jv"]
MPM_NOALLOC_SCRATCH_BYTES = 32 << 20

_lib = None


def load():
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "mpm_create": ([C.POINTER(P), C.c_int, P], C.c_int),
        "mpm_destroy": ([P], C.c_int),
        "mpm_last_error": ([P], C.c_char_p),
        "mpm_prepare": ([P, C.POINTER(mpm_problem), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                         C.POINTER(C.c_int32)], C.c_int),
        "mpm_residual": ([P, C.POINTER(mpm_problem), P, P, P, C.POINTER(C.c_double)], C.c_int),
        "mpm_residual_noalloc": ([P, C.POINTER(mpm_problem), P, P, P, C.POINTER(C.c_double)], C.c_int),
        "mpm_jacobian_bsr": ([P, C.POINTER(mpm_problem), P, P, P, P, P, C.c_int32], C.c_int),
        "mpm_newton_step": ([P, C.POINTER(mpm_problem), C.POINTER(mpm_newton_opts), P,
                             C.POINTER(mpm_newton_report)], C.c_int),
        "mpm_update": ([P, C.POINTER(mpm_problem), P, P, P, P], C.c_int),
        "mpm_spmv": ([P, P, P, P, P], C.c_int),
        "mpm_jv": ([P, C.POINTER(mpm_problem), P, P, P, C.c_int32], C.c_int),
        "mpm_spmv_lanes": ([P], C.c_int),
        "mpm_spmv_set_lanes": ([P, C.c_int32], C.c_int),
        "mpm_adjoint_step": ([P, C.POINTER(mpm_problem), P, C.POINTER(C.c_double), P, P, P, C.c_double,
                              C.POINTER(C.c_int32), C.POINTER(C.c_double)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(ctx, rc):
    if rc != MPM_OK:
        msg = load().mpm_last_error(ctx).decode() if ctx else ""
        raise MPMError(rc, msg)


# ------------------------------------------------------------ problem ------
@dataclass
class DeviceProblem:
    """Device tensors of one load step (one or several sims) and the C struct
    pointing at them.  Keep the object alive while the library uses it."""
    struct: mpm_problem
    tensors: dict
    grids: object
    sim_start: object
    dim: int
    ndof: int
    nsim: int
    np_per_sim: list
    nodes_per_sim: list


def make_problem(sims, bcs, device="cuda", react_masks=None) -> DeviceProblem:
    """Build the device problem from host workloads.

    sims: list of (Problem, Particles) from ``workloads``; bcs: list of
    Dirichlet; react_masks: list of uint8 arrays [n_nodes][ndof] or None.
    All sims must share dim and the material constants except E and phi.
    """
    import torch
    P0 = sims[0][0]
    dim, nd, nsim = P0.dim, P0.ndof, len(sims)
    per_particle = nsim > 1 or any(st.E is not None or st.phi is not None for _, st in sims)

    def cat(field, ncomp):
        arrs = [getattr(st, field) for _, st in sims]
        if any(a is None for a in arrs):
            return None
        return np.ascontiguousarray(np.concatenate([np.asarray(a).reshape(ncomp, -1) for a in arrs], axis=1))

    x = cat("x", dim)
    vol0 = np.concatenate([st.vol0 for _, st in sims])
    F = cat("F", dim * dim)
    be = cat("be", 4 if dim == 2 else 6)
    fp = cat("fp", dim) if all(st.fp is not None for _, st in sims) else None
    if per_particle:
        E = np.concatenate([st.E if st.E is not None else np.full(st.np, p.E) for p, st in sims])
        phi = np.concatenate([st.phi if st.phi is not None else np.full(st.np, p.phi) for p, st in sims])
    else:
        E = phi = None
    mask = np.concatenate([b.mask.reshape(-1) for b in bcs]).astype(np.uint8)
    value = np.concatenate([b.value.reshape(-1) for b in bcs]).astype(np.float64)
    react = None
    if react_masks is not None:
        react = np.concatenate([m.reshape(-1) for m in react_masks]).astype(np.uint8)

    td = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
    T = {"x": td(x), "vol0": td(vol0), "F": td(F), "be": td(be), "fp": td(fp), "E": td(E), "phi": td(phi),
         "bc_mask": td(mask), "bc_value": td(value), "react": td(react)}

    grids = (mpm_grid * nsim)()
    for s, (p, _) in enumerate(sims):
        grids[s].dim = dim
        for k in range(3):
            grids[s].ncell[k] = int(p.n[k]) if k < dim else 0
            grids[s].origin[k] = float(p.x0[k]) if k < dim else 0.0
        grids[s].h = float(p.h)
    nps = [st.np for _, st in sims]
    ss = (C.c_int64 * (nsim + 1))(*np.concatenate([[0], np.cumsum(nps)]).astype(np.int64).tolist())

    m = mpm_material()
    m.up, m.dp, m.dp_match = int(P0.up), int(P0.dp), int(P0.dp_match)
    m.E, m.nu, m.phi, m.c, m.psi = P0.E, P0.nu, P0.phi, P0.c, P0.psi
    m.rho0 = P0.rho0
    for k in range(3):
        m.g[k] = float(P0.g[k]) if k < len(P0.g) else 0.0
    m.perm, m.mu_f, m.biot, m.rho_f, m.dt = P0.perm, P0.mu_f, P0.biot, P0.rho_f, P0.dt
    m.apex_reg = float(getattr(P0, "apex_reg", 0.0))
    m.shape = int(getattr(P0, "shape", 0))
    m.elastic = int(getattr(P0, "elastic", 0))
    lp0 = getattr(P0, "lp0", (0.0, 0.0, 0.0))
    for k in range(3):
        m.lp0[k] = float(lp0[k]) if k < len(lp0) else 0.0

    pr = mpm_problem()
    pr.nsim = nsim
    pr.grids = grids
    pr.sim_start = ss if nsim > 1 else None
    pr.mat = m
    pr.P = mpm_particles(int(vol0.shape[0]), _ptr(T["x"]), _ptr(T["vol0"]), _ptr(T["F"]), _ptr(T["be"]),
                         _ptr(T["fp"]), _ptr(T["E"]), _ptr(T["phi"]))
    pr.bc_mask = _ptr(T["bc_mask"])
    pr.bc_value = _ptr(T["bc_value"])
    pr.react_mask = _ptr(T["react"])
    return DeviceProblem(pr, T, grids, ss, dim, nd, nsim, nps, [p.n_nodes for p, _ in sims])


def set_bc(dp: DeviceProblem, bcs):
    """Replace the Dirichlet data in place (same shapes)."""
    import torch
    mask = np.concatenate([b.mask.reshape(-1) for b in bcs]).astype(np.uint8)
    value = np.concatenate([b.value.reshape(-1) for b in bcs]).astype(np.float64)
    dp.tensors["bc_mask"].copy_(torch.from_numpy(mask))
    dp.tensors["bc_value"].copy_(torch.from_numpy(value))


# ----------------------------------------------------- C-ABI functions -----
def mpm_create(device=0, stream=None):
    import torch
    lib = load()
    ctx = C.c_void_p()
    if stream is None:
        stream = torch.cuda.current_stream(device).cuda_stream
    rc = lib.mpm_create(C.byref(ctx), int(device), C.c_void_p(stream))
    if rc != MPM_OK:
        raise MPMError(rc, "mpm_create failed")
    return ctx


def mpm_destroy(ctx):
    load().mpm_destroy(ctx)


def mpm_prepare(ctx, dp: DeviceProblem):
    n_row, nnzb, nd = C.c_int64(), C.c_int64(), C.c_int32()
    _check(ctx, load().mpm_prepare(ctx, C.byref(dp.struct), C.byref(n_row), C.byref(nnzb), C.byref(nd)))
    return n_row.value, nnzb.value, nd.value


def mpm_residual(ctx, dp: DeviceProblem, du, r, r_raw=None, want_reaction=False):
    react = (C.c_double * dp.nsim)() if want_reaction else None
    _check(ctx, load().mpm_residual(ctx, C.byref(dp.struct), _ptr(du), _ptr(r), _ptr(r_raw),
                                    react if react is not None else None))
    return None if react is None else np.array(react[:])


def mpm_residual_noalloc(ctx, dp: DeviceProblem, du, r, r_raw=None, want_reaction=False):
    react = (C.c_double * dp.nsim)() if want_reaction else None
    _check(ctx, load().mpm_residual_noalloc(ctx, C.byref(dp.struct), _ptr(du), _ptr(r), _ptr(r_raw),
                                            react if react is not None else None))
    return None if react is None else np.array(react[:])


def mpm_jacobian_bsr(ctx, dp: DeviceProblem, du, rowptr=None, colind=None, val=None, active_nodes=None, raw=False):
    _check(ctx, load().mpm_jacobian_bsr(ctx, C.byref(dp.struct), _ptr(du), _ptr(rowptr), _ptr(colind), _ptr(val),
                                        _ptr(active_nodes), MPM_JAC_RAW if raw else 0))


def mpm_newton_step(ctx, dp: DeviceProblem, du, tol=1e-10, max_iter=25, commit=True, stall_factor=1e3,
                    krylov_rtol=1e-12, krylov_max_iter=20000, line_search=0, time_spmv=0, krylov_method=0,
                    raise_on_fail=True):
    o = mpm_newton_opts(tol, max_iter, 1 if commit else 0, stall_factor, krylov_rtol, krylov_max_iter,
                        int(line_search), int(time_spmv), int(krylov_method))
    rep = mpm_newton_report()
    it = (C.c_int32 * dp.nsim)()
    cv = (C.c_int32 * dp.nsim)()
    re = (C.c_double * dp.nsim)()
    rl = (C.c_double * dp.nsim)()
    rep.sim_iters, rep.sim_converged, rep.sim_reaction, rep.sim_rel = it, cv, re, rl
    rc = load().mpm_newton_step(ctx, C.byref(dp.struct), C.byref(o), _ptr(du), C.byref(rep))
    out = {"status": rc, "iters": rep.iters, "converged": bool(rep.converged), "krylov_iters": rep.krylov_iters,
           "norms": list(rep.norms[:max(1, min(rep.iters + 1, MPM_MAX_REPORT))]),
           "krylov": list(rep.krylov[:max(0, min(rep.iters, MPM_MAX_REPORT))]),
           "ms_residual": rep.ms_residual, "ms_jacobian": rep.ms_jacobian, "ms_krylov": rep.ms_krylov,
           "ms_total": rep.ms_total, "spmv_ms": rep.spmv_ms, "spmv_launches": rep.spmv_launches,
           "sim_iters": list(it), "sim_converged": list(cv), "sim_reaction": list(re), "sim_rel": list(rl),
           "precond_flags": rep.precond_flags}
    if rc != MPM_OK and raise_on_fail:
        _check(ctx, rc)
    return out


def mpm_update(ctx, dp: DeviceProblem, du, x_out, F_out, be_out):
    _check(ctx, load().mpm_update(ctx, C.byref(dp.struct), _ptr(du), _ptr(x_out), _ptr(F_out), _ptr(be_out)))


MPM_JV_REUSE = 2


def mpm_jv(ctx, dp: DeviceProblem, du, x, y, raw=False, reuse=False):
    flags = (MPM_JAC_RAW if raw else 0) | (MPM_JV_REUSE if reuse else 0)
    _check(ctx, load().mpm_jv(ctx, C.byref(dp.struct), _ptr(du), _ptr(x), _ptr(y), flags))


def mpm_spmv(ctx, val, x, y, z=None):
    _check(ctx, load().mpm_spmv(ctx, _ptr(val), _ptr(x), _ptr(y), _ptr(z)))


def mpm_spmv_lanes(ctx):
    """Lanes per BSR row the SpMV autotuner picked (0 before the first product)."""
    return int(load().mpm_spmv_lanes(ctx))


def mpm_spmv_set_lanes(ctx, lanes):
    """Pin the SpMV launch shape (4, 8, 16 lanes per row; 0: autotune).
    Results do not depend on it."""
    _check(ctx, load().mpm_spmv_set_lanes(ctx, int(lanes)))


def mpm_adjoint_step(ctx, dp: DeviceProblem, du, react_bar, sbar_next, sbar_n, theta_bar, krylov_rtol=1e-12,
                     with_rel=False):
    """One step's adjoint; react_bar is a host sequence [nsim].  Returns the
    Krylov iterations of the transposed solve per sim (and, with with_rel,
    the true relative residual each sim's solve reached)."""
    rb = (C.c_double * dp.nsim)(*[float(v) for v in react_bar])
    it = (C.c_int32 * dp.nsim)()
    rl = (C.c_double * dp.nsim)()
    _check(ctx, load().mpm_adjoint_step(ctx, C.byref(dp.struct), _ptr(du), rb, _ptr(sbar_next), _ptr(sbar_n),
                                        _ptr(theta_bar), float(krylov_rtol), it, rl))
    return (list(it), list(rl)) if with_rel else list(it)
