"""Python driver for the plain FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use this module. It never imports the product package and the
product package never imports it.

The numerical work sits in ``mpm_oracle.cpp`` (residual, local dual-number
Jacobians, particle update).  This file adds what the paper leaves to a
driver:

* the Jacobian sparsity pattern by brute force (every occupied stencil
  contributes all of its node pairs; Sec. 3.2, the block-sparse structure
  with at most 5^d coupled nodes per node, Table 1);
* Dirichlet handling and the Newton iteration of Sec. 2.2 (solve
  -J du = r, stop on ||r_k|| / ||r_0|| <= tol), with SciPy's sparse direct
  solver standing in for the paper's linear solvers (Remark 2).

A "problem" here is any object with the attributes listed in ``_cfg`` and a
"state" any object with ``x, vol0, F, be, fp, E, phi`` arrays (``fp``, ``E``
and ``phi`` may be None).  Vectors over the grid are "full" (every node of
the padded grid, nodes -1..n+1 per axis, x fastest, node-interleaved
unknowns) unless named "compact" (active rows only).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpm_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [("dim", C.c_int32), ("up", C.c_int32), ("dp", C.c_int32), ("dp_match", C.c_int32),
                ("n", C.c_int32 * 3), ("h", C.c_double), ("x0", C.c_double * 3),
                ("E", C.c_double), ("nu", C.c_double), ("phi", C.c_double), ("c", C.c_double),
                ("psi", C.c_double), ("rho0", C.c_double), ("g", C.c_double * 3),
                ("perm", C.c_double), ("mu_f", C.c_double), ("biot", C.c_double),
                ("rho_f", C.c_double), ("dt", C.c_double), ("apex_reg", C.c_double),
                ("shape", C.c_int32), ("pad_", C.c_int32), ("lp0", C.c_double * 3),
                ("elastic", C.c_int32), ("pad2_", C.c_int32)]


class _Particles(C.Structure):
    _fields_ = [("np", C.c_int64), ("x", C.c_void_p), ("vol0", C.c_void_p), ("F", C.c_void_p),
                ("be", C.c_void_p), ("fp", C.c_void_p), ("E", C.c_void_p), ("phi", C.c_void_p)]


class _Tangents(C.Structure):
    _fields_ = [("x", C.c_void_p), ("F", C.c_void_p), ("be", C.c_void_p), ("theta", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        for name, args in [
            ("orc_forces", [P, P, P, P, P, P]),
            ("orc_node_volume", [P, P, P]),
            ("orc_origins", [P, P, P]),
            ("orc_jacobian_bsr", [P, P, P, P, P, P, P]),
            ("orc_dense_jacobian", [P, P, P, P]),
            ("orc_update", [P, P, P, P, P, P]),
            ("orc_stress", [P, P, P, P, P]),
            ("orc_logm", [P, P]), ("orc_expm", [P, P]), ("orc_logm_dir", [P, P, P, P]),
            ("orc_return_map", [P, C.c_double, C.c_double, P, P, P]),
            ("orc_return_map_dir", [P, C.c_double, C.c_double, P, P, P, P]),
            ("orc_bspline", [C.c_double, C.c_int64, P, P]),
            ("orc_gimp", [C.c_double, C.c_int64, C.c_double, P, P]),
            ("orc_forces_tan", [P, P, P, P, P, P, P, P, P]),
            ("orc_update_tan", [P, P, P, P, P, P, P, P, P, P, P]),
        ]:
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def cfg(prob) -> _Cfg:
    c = _Cfg()
    c.dim, c.up, c.dp, c.dp_match = prob.dim, int(prob.up), int(prob.dp), int(prob.dp_match)
    for k in range(3):
        c.n[k] = int(prob.n[k]) if k < len(prob.n) else 0
        c.x0[k] = float(prob.x0[k]) if k < len(prob.x0) else 0.0
        c.g[k] = float(prob.g[k]) if k < len(prob.g) else 0.0
    c.h = float(prob.h)
    c.E, c.nu, c.phi, c.c, c.psi = (float(v) for v in (prob.E, prob.nu, prob.phi, prob.c, prob.psi))
    c.rho0, c.perm, c.mu_f, c.biot, c.rho_f, c.dt = (float(v) for v in (
        prob.rho0, prob.perm, prob.mu_f, prob.biot, prob.rho_f, prob.dt))
    c.apex_reg = float(getattr(prob, "apex_reg", 0.0))
    c.shape = int(getattr(prob, "shape", 0))
    c.elastic = int(getattr(prob, "elastic", 0))
    lp0 = getattr(prob, "lp0", (0.0, 0.0, 0.0))
    for k in range(3):
        c.lp0[k] = float(lp0[k]) if k < len(lp0) else 0.0
    return c


class _PartRef:
    """Keeps the contiguous copies alive while C holds their pointers."""

    def __init__(self, st):
        self.arrs = [_c64(st.x), _c64(st.vol0), _c64(st.F), _c64(st.be), _c64(st.fp),
                     _c64(st.E), _c64(st.phi)]
        self.s = _Particles(int(self.arrs[1].shape[0]), *[_ptr(a) for a in self.arrs])


def ndof(prob) -> int:
    return prob.dim + (1 if prob.up else 0)


def nodes_per_axis(prob):
    return [int(prob.n[k]) + 3 for k in range(prob.dim)]


def n_nodes(prob) -> int:
    return int(np.prod(nodes_per_axis(prob)))


# ----------------------------------------------------------------- forces --
def forces(prob, st, dof_full):
    """Internal and external nodal forces, full grid, shape (n_nodes, ndof)."""
    nd = ndof(prob)
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    fint = np.zeros(n_nodes(prob) * nd)
    fext = np.zeros(n_nodes(prob) * nd)
    c, P = cfg(prob), _PartRef(st)
    lib().orc_forces(C.byref(c), C.byref(P.s), _ptr(dof), _ptr(fint), _ptr(fext), None)
    return fint.reshape(-1, nd), fext.reshape(-1, nd)


def regimes(prob, st, dof_full):
    nd = ndof(prob)
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    fint = np.zeros(n_nodes(prob) * nd)
    reg = np.zeros(st.vol0.shape[0], dtype=np.int32)
    c, P = cfg(prob), _PartRef(st)
    lib().orc_forces(C.byref(c), C.byref(P.s), _ptr(dof), _ptr(fint), None, _ptr(reg))
    return reg


def stress(prob, st, dof_full):
    """Kirchhoff stress (np, 3, 3) and regime per particle at the given unknowns."""
    np_ = st.vol0.shape[0]
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    tau = np.zeros(9 * np_)
    reg = np.zeros(np_, dtype=np.int32)
    c, P = cfg(prob), _PartRef(st)
    lib().orc_stress(C.byref(c), C.byref(P.s), _ptr(dof), _ptr(tau), _ptr(reg))
    return tau.reshape(3, 3, np_).transpose(2, 0, 1), reg


def node_volume(prob, st):
    out = np.zeros(n_nodes(prob))
    c, P = cfg(prob), _PartRef(st)
    lib().orc_node_volume(C.byref(c), C.byref(P.s), _ptr(out))
    return out


def origins(prob, st):
    np_ = st.vol0.shape[0]
    o = np.zeros(prob.dim * np_, dtype=np.int64)
    c, P = cfg(prob), _PartRef(st)
    lib().orc_origins(C.byref(c), C.byref(P.s), _ptr(o))
    return o.reshape(prob.dim, np_)


# ---------------------------------------------------------------- pattern --
@dataclass
class Pattern:
    active: np.ndarray       # int64 full-grid node ids of the rows, ascending
    rowptr: np.ndarray       # int32 [n_row + 1]
    colind: np.ndarray       # int32 [nnzb], ascending within a row
    row_of_node: np.ndarray  # int64 [n_nodes], -1 where inactive

    @property
    def n_row(self):
        return int(self.active.shape[0])

    @property
    def nnzb(self):
        return int(self.colind.shape[0])


def pattern(prob, st) -> Pattern:
    """Brute force: every occupied stencil origin couples all pairs of its
    3^d nodes; rows are active nodes in ascending linear order."""
    d = prob.dim
    npa = np.array(nodes_per_axis(prob), dtype=np.int64)
    o = origins(prob, st)                                   # [d][np]
    # linear origin id on the node lattice (origin -1 -> 0)
    strides = np.cumprod(np.concatenate([[1], npa[:-1]]))
    lin = ((o + 1) * strides[:, None]).sum(axis=0)
    uo = np.unique(lin)
    offs = np.array(np.meshgrid(*[np.arange(3)] * d, indexing="ij")).reshape(d, -1)  # [d][3^d]
    offs_lin = (offs * strides[:, None]).sum(axis=0)
    nodes = uo[:, None] + offs_lin[None, :]                 # [n_origin][3^d]
    active = np.unique(nodes)
    nn = n_nodes(prob)
    row_of_node = np.full(nn, -1, dtype=np.int64)
    row_of_node[active] = np.arange(active.shape[0])
    k = nodes.shape[1]
    ri = np.repeat(nodes, k, axis=1).reshape(-1)
    ci = np.tile(nodes, (1, k)).reshape(-1)
    key = np.unique(row_of_node[ri] * active.shape[0] + row_of_node[ci])
    rows = key // active.shape[0]
    cols = key % active.shape[0]
    rowptr = np.zeros(active.shape[0] + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return Pattern(active.astype(np.int64), rowptr.astype(np.int32), cols.astype(np.int32), row_of_node)


def jacobian_bsr(prob, st, dof_full, pat: Pattern):
    """Raw Jacobian d f_int / d unknowns in the BSR pattern, values
    [nnzb][ndof][ndof] (no Dirichlet rows applied)."""
    nd = ndof(prob)
    val = np.zeros(pat.nnzb * nd * nd)
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    c, P = cfg(prob), _PartRef(st)
    rc = lib().orc_jacobian_bsr(C.byref(c), C.byref(P.s), _ptr(dof), _ptr(pat.row_of_node),
                                _ptr(pat.rowptr), _ptr(pat.colind), _ptr(val))
    if rc != 0:
        raise RuntimeError("oracle: particle block outside the pattern")
    return val.reshape(pat.nnzb, nd, nd)


def dense_jacobian(prob, st, dof_full):
    nd = ndof(prob)
    ntot = n_nodes(prob) * nd
    out = np.zeros(ntot * ntot)
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    c, P = cfg(prob), _PartRef(st)
    lib().orc_dense_jacobian(C.byref(c), C.byref(P.s), _ptr(dof), _ptr(out))
    return out.reshape(ntot, ntot)


def bsr_to_dense(pat: Pattern, val, nd):
    n = pat.n_row * nd
    A = np.zeros((n, n))
    for r in range(pat.n_row):
        for b in range(pat.rowptr[r], pat.rowptr[r + 1]):
            cidx = pat.colind[b]
            A[r * nd:(r + 1) * nd, cidx * nd:(cidx + 1) * nd] = val[b]
    return A


def bsr_to_scipy(pat: Pattern, val, nd):
    import scipy.sparse as sp
    n = pat.n_row * nd
    return sp.bsr_matrix((val, pat.colind.astype(np.int64), pat.rowptr.astype(np.int64)), shape=(n, n)).tocsr()


# ------------------------------------------------------------------ state --
@dataclass
class State:
    x: np.ndarray
    vol0: np.ndarray
    F: np.ndarray
    be: np.ndarray
    fp: np.ndarray | None = None
    E: np.ndarray | None = None
    phi: np.ndarray | None = None

    def copy(self):
        cp = lambda a: None if a is None else a.copy()
        return State(cp(self.x), cp(self.vol0), cp(self.F), cp(self.be), cp(self.fp), cp(self.E), cp(self.phi))


def update(prob, st, dof_full):
    """End-of-step particle update; returns a new State."""
    new = st.copy()
    new.x = np.ascontiguousarray(new.x); new.F = np.ascontiguousarray(new.F); new.be = np.ascontiguousarray(new.be)
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    c, P = cfg(prob), _PartRef(st)
    lib().orc_update(C.byref(c), C.byref(P.s), _ptr(dof), _ptr(new.x), _ptr(new.F), _ptr(new.be))
    return new


# ----------------------------------------------------------------- Newton --
@dataclass
class NewtonReport:
    iters: int
    norms: list
    converged: bool
    reaction: np.ndarray | None = None


def constrained(prob, st, pat: Pattern, mask_full):
    """Compact (n_row, ndof) boolean mask of constrained unknowns; nodes
    without material (zero weight sum) are constrained in every unknown."""
    m = np.asarray(mask_full, dtype=bool).reshape(-1, ndof(prob))[pat.active].copy()
    vol = node_volume(prob, st)[pat.active]
    m[vol == 0.0, :] = True
    return m


def apply_dirichlet(A, cmask_flat):
    import scipy.sparse as sp
    free = (~cmask_flat).astype(np.float64)
    D = sp.diags(free)
    return (D @ A @ D + sp.diags(1.0 - free)).tocsr()


def _field_norms(prob, r):
    """One 2-norm over every free unknown, as in the paper's stopping rule
    (Sec. 2.2); for u-p the vector holds both fields."""
    return [float(np.linalg.norm(r))]


def newton(prob, st, mask_full, value_full, tol=1e-10, maxit=25, dof0_full=None, pat=None,
           reaction_nodes=None, reaction_dof=None, solver="direct", stall_factor=1e3, line_search=0):
    """Newton iteration for one load step (Sec. 2.2).

    Unknowns start at ``dof0_full`` (zero if None) with the constrained ones
    set to ``value_full``.  Stops when ||r_k|| / ||r_0|| <= tol over the free
    unknowns, or when it stalls at the FP64 round-off floor: ||r_k|| <=
    stall_factor * tol * ||r_0|| and ||r_k|| > ||r_{k-1}|| / 2.
    Returns (dof_full, report, pattern)."""
    import scipy.sparse.linalg as spla
    nd = ndof(prob)
    if pat is None:
        pat = pattern(prob, st)
    mask_full = np.asarray(mask_full, dtype=bool).reshape(-1, nd)
    dof = np.zeros((n_nodes(prob), nd)) if dof0_full is None else np.array(dof0_full, dtype=np.float64).reshape(-1, nd)
    dof[mask_full] = np.asarray(value_full).reshape(-1, nd)[mask_full]
    cm = constrained(prob, st, pat, mask_full)
    vol = node_volume(prob, st)[pat.active]
    dof[pat.active[vol == 0.0]] = 0.0
    norms, norm0 = [], None
    reaction = None
    converged = False
    it = 0
    for it in range(maxit + 1):
        fint, fext = forces(prob, st, dof)
        rfull = fint - fext
        if reaction_nodes is not None:
            reaction = -rfull[reaction_nodes, reaction_dof].sum()
        r = rfull[pat.active].copy()
        r[cm] = 0.0
        nrm = _field_norms(prob, r)
        norms.append(nrm)
        if norm0 is None:
            norm0 = [max(v, 1e-300) for v in nrm]
        # converged: relative drop reached, or stalled at the FP64 floor
        # (within stall_factor * tol of r_0 and no longer halving)
        prev = norms[-2] if len(norms) > 1 else None
        if all(v <= tol * n0 or v == 0.0 for v, n0 in zip(nrm, norm0)) or (
                prev is not None and all(v <= stall_factor * tol * n0 and v > 0.5 * pv
                                         for v, n0, pv in zip(nrm, norm0, prev))):
            converged = True
            break
        if it == maxit:
            break
        val = jacobian_bsr(prob, st, dof, pat)
        A = apply_dirichlet(bsr_to_scipy(pat, val, nd), cm.reshape(-1))
        rhs = -r.reshape(-1)
        if solver == "direct":
            delta = spla.spsolve(A.tocsc(), rhs)
        else:
            delta = _bicgstab_bj(A, rhs, nd)
        step = delta.reshape(-1, nd)
        alpha = 1.0
        if line_search:
            # backtracking on the residual norm: halve the step until
            # ||r(u + a d)|| < (1 - 1e-4 a) ||r(u)||
            base = dof.copy()
            for _ in range(line_search):
                dof[pat.active] = base[pat.active] + alpha * step
                fi2, fe2 = forces(prob, st, dof)
                r2 = (fi2 - fe2)[pat.active]
                r2[cm] = 0.0
                if np.linalg.norm(r2) < (1.0 - 1e-4 * alpha) * nrm[0]:
                    break
                alpha *= 0.5
            else:
                dof[pat.active] = base[pat.active] + step
        else:
            dof[pat.active] += step
    return dof, NewtonReport(it, norms, converged, reaction), pat


def _bicgstab_bj(A, b, nd, rtol=1e-12, maxiter=20000):
    """SciPy BiCGStab with a block-Jacobi preconditioner (for large grids)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = A.shape[0] // nd
    blocks = np.zeros((n, nd, nd))
    Ad = A.tocoo()
    sel = (Ad.row // nd) == (Ad.col // nd)
    blocks[Ad.row[sel] // nd, Ad.row[sel] % nd, Ad.col[sel] % nd] = Ad.data[sel]
    inv = np.linalg.inv(blocks)
    M = sp.block_diag(list(inv), format="csr") if n < 2000 else _block_diag_csr(inv)
    x, info = spla.bicgstab(A, b, rtol=rtol, atol=0.0, maxiter=maxiter, M=M)
    if info != 0:
        raise RuntimeError(f"oracle BiCGStab did not converge (info={info})")
    return x


def _block_diag_csr(inv):
    import scipy.sparse as sp
    n, nd, _ = inv.shape
    indptr = np.arange(n + 1) * 1
    return sp.bsr_matrix((inv, np.arange(n), indptr), shape=(n * nd, n * nd)).tocsr()


# ------------------------------------------------- forward sensitivity -----
@dataclass
class StateTangent:
    """Tangents of the particle state in two directions (E, phi)."""
    x: np.ndarray     # [2][dim][np]
    F: np.ndarray     # [2][dim*dim][np]
    be: np.ndarray    # [2][nb][np]

    @staticmethod
    def zeros(dim, np_):
        nb = 4 if dim == 2 else 6
        return StateTangent(np.zeros((2, dim, np_)), np.zeros((2, dim * dim, np_)), np.zeros((2, nb, np_)))


_THETA = np.ascontiguousarray(np.eye(2))   # direction 0 seeds E, direction 1 seeds phi


def _tan_struct(tan):
    arrs = [np.ascontiguousarray(tan.x), np.ascontiguousarray(tan.F), np.ascontiguousarray(tan.be), _THETA]
    return arrs, _Tangents(*[_ptr(a) for a in arrs])


def forces_tan(prob, st, tan, dof_full, dof_t):
    """f_int, f_ext and their tangents [2][n_nodes][ndof] (full grid)."""
    nd = ndof(prob)
    nn = n_nodes(prob) * nd
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    dt = np.ascontiguousarray(dof_t, dtype=np.float64).reshape(-1)
    fi, fe = np.zeros(nn), np.zeros(nn)
    fit, fet = np.zeros(2 * nn), np.zeros(2 * nn)
    c, P = cfg(prob), _PartRef(st)
    keep, T = _tan_struct(tan)
    lib().orc_forces_tan(C.byref(c), C.byref(P.s), C.byref(T), _ptr(dof), _ptr(dt), _ptr(fi), _ptr(fe), _ptr(fit),
                         _ptr(fet))
    return fi.reshape(-1, nd), fe.reshape(-1, nd), fit.reshape(2, -1, nd), fet.reshape(2, -1, nd)


def update_tan(prob, st, tan, dof_full, dof_t):
    new = st.copy()
    new.x = np.ascontiguousarray(new.x); new.F = np.ascontiguousarray(new.F); new.be = np.ascontiguousarray(new.be)
    nt = StateTangent.zeros(prob.dim, st.vol0.shape[0])
    dof = np.ascontiguousarray(dof_full, dtype=np.float64).reshape(-1)
    dt = np.ascontiguousarray(dof_t, dtype=np.float64).reshape(-1)
    c, P = cfg(prob), _PartRef(st)
    keep, T = _tan_struct(tan)
    lib().orc_update_tan(C.byref(c), C.byref(P.s), C.byref(T), _ptr(dof), _ptr(dt), _ptr(new.x), _ptr(new.F),
                         _ptr(new.be), _ptr(nt.x), _ptr(nt.F), _ptr(nt.be))
    return new, nt


def simulate_sensitivity(prob, st0, bcs, react_nodes, react_dof, tol=1e-12, line_search=0):
    """Run load steps with Newton and carry forward sensitivities of the
    reaction to the two material parameters (E, phi) shared by all particles.

    Per step: converged du; the tangent d(du)/d(theta) solves
    J d(du) = -(dr/ds . ds/dtheta + dr/dtheta) on the free unknowns (the
    implicit function of r(du; s, theta) = 0); the reaction and the state
    update are then differentiated along (d(du), ds, e_theta).
    Returns (reactions [n_steps], dR/dtheta [n_steps][2], final state)."""
    import scipy.sparse.linalg as spla
    nd = ndof(prob)
    st = st0.copy()
    tan = StateTangent.zeros(prob.dim, st.vol0.shape[0])
    R, dR = [], []
    for bc in bcs:
        dof, rep, pat = newton(prob, st, bc.mask, bc.value, tol=tol, line_search=line_search)
        if not rep.converged:
            raise RuntimeError("oracle Newton did not converge in the sensitivity run")
        cm = constrained(prob, st, pat, bc.mask)
        A = apply_dirichlet(bsr_to_scipy(pat, jacobian_bsr(prob, st, dof, pat), nd), cm.reshape(-1)).tocsc()
        zero_t = np.zeros((2, n_nodes(prob), nd))
        _, _, fit, fet = forces_tan(prob, st, tan, dof, zero_t)
        ddu = np.zeros((2, n_nodes(prob), nd))
        for k in range(2):
            rt = (fit[k] - fet[k])[pat.active]
            rt[cm] = 0.0
            ddu[k][pat.active] = spla.spsolve(A, -rt.reshape(-1)).reshape(-1, nd)
        fi, fe, fit, fet = forces_tan(prob, st, tan, dof, ddu)
        R.append(-(fi - fe)[react_nodes, react_dof].sum())
        dR.append([-(fit[k] - fet[k])[react_nodes, react_dof].sum() for k in range(2)])
        st, tan = update_tan(prob, st, tan, dof, ddu)
    return np.array(R), np.array(dR), st
