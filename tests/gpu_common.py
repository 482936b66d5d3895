"""Helpers shared by the GPU parity tests: run a workload through the C ABI
and through the oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2507_09435_amd import mpm as M
from paper_2507_09435_amd import workloads as W


def react_mask(w: W.Workload):
    P = w.prob
    m = np.zeros((P.n_nodes, P.ndof), dtype=np.uint8)
    if w.footing is not None:
        m[w.footing_nodes(), w.footing[1]] = 1
    return m


def oracle_pattern_batch(sims):
    """Concatenate per-sim oracle patterns with node and row offsets."""
    act, rp, ci = [], [0], []
    node_off = row_off = 0
    pats = []
    for P, st in sims:
        pat = O.pattern(P, st)
        pats.append(pat)
        act.append(pat.active + node_off)
        rp.extend((pat.rowptr[1:] + rp[-1]).tolist())
        ci.append(pat.colind + row_off)
        node_off += P.n_nodes
        row_off += pat.n_row
    return np.concatenate(act), np.array(rp, dtype=np.int64), np.concatenate(ci), pats


def compact_to_full(P, pat, v):
    full = np.zeros((P.n_nodes, P.ndof))
    full[pat.active] = np.asarray(v).reshape(-1, P.ndof)
    return full


def seeded_du(P, pat, seed, amp=2e-3):
    rng = np.random.default_rng(seed)
    du = rng.normal(size=(pat.n_row, P.ndof)) * amp * P.h
    du[:, 1] -= amp * P.h
    if P.up:
        du[:, P.dim] = rng.normal(size=pat.n_row) * 1e3
    return du


def rel_err(a, b, scale=None):
    a, b = np.asarray(a), np.asarray(b)
    s = np.linalg.norm(b) if scale is None else scale
    return np.linalg.norm(a - b) / max(s, 1e-300)


def row_errors(got, ref, fint, fext):
    """Per row: ||r_gpu - r_ref|| / (||f_int,row|| + ||f_ext,row|| + 1e-12 max over rows of both)
    (rows whose forces all vanish, as where a node's weight is exactly zero, count as 0 / tiny)."""
    g, r = np.asarray(got).reshape(ref.shape), np.asarray(ref)
    fi, fe = np.linalg.norm(fint, axis=1), np.linalg.norm(fext, axis=1)
    return np.linalg.norm(g - r, axis=1) / (fi + fe + 1e-12 * max(fi.max(), fe.max()) + 1e-300)


def block_errors(val_gpu, val_ref):
    """Per-block ||B_gpu - B_ref||_F / max(||B_ref||_F, 1e-12 max ||B_ref||_F)."""
    nb = val_ref.shape[0]
    g = val_gpu.reshape(nb, -1)
    r = val_ref.reshape(nb, -1)
    nr = np.linalg.norm(r, axis=1)
    floor = 1e-12 * nr.max()
    return np.linalg.norm(g - r, axis=1) / np.maximum(nr, floor)


def dirichlet_bsr(pat, val, cm):
    """Zero constrained rows and columns of BSR blocks, 1 on the diagonal."""
    out = np.array(val, copy=True)
    rows = np.repeat(np.arange(pat.n_row), np.diff(pat.rowptr))
    for k in range(pat.nnzb):
        r, c = rows[k], pat.colind[k]
        for i in range(out.shape[1]):
            for j in range(out.shape[2]):
                if cm[r, i] or cm[c, j]:
                    out[k, i, j] = 1.0 if (r == c and i == j) else 0.0
    return out
