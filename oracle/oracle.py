"""ctypes front end of the C oracle (sgp_oracle.c).

TEST INFRASTRUCTURE ONLY.  The functions return plain numpy arrays; they
mirror the steps of the method one to one:

  collide -> assemble -> prim (or kruskal) -> root_forest -> tree_order
          -> tree_factor -> tree_solve / pcg / ir_solve

Defaults are the friction constants of the synthetic workloads: g_par = 1,
g_perp = 0.1, g_med = 1e-3.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

G_PAR, G_PERP, G_MED = 1.0, 0.1, 1e-3

OK, EINVAL, ENOMEM, ENOTSPD, ENOCONV, EBREAKDOWN, ENONFINITE = 0, -1, -2, -5, -6, -7, -8
PREC = {"none": 0, "jacobi": 1, "tree": 2}

_lib = None


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64),
                ("rowptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("ei", C.POINTER(C.c_int32)), ("ej", C.POINTER(C.c_int32)),
                ("w", C.POINTER(C.c_double)), ("u", C.POINTER(C.c_double))]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        L.orc_collide_brute.restype = C.POINTER(_Graph)
        L.orc_collide_cells.restype = C.POINTER(_Graph)
        for f in ("orc_prim", "orc_kruskal"):
            getattr(L, f).restype = C.c_int64
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _i32(a):
    return _p(a, C.c_int32)


def _f64(a):
    return _p(a, C.c_double)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


@dataclass
class Graph:
    n: int
    rowptr: np.ndarray  # int32 [n+1]
    col: np.ndarray     # int32 [2m]
    ei: np.ndarray      # int32 [m]
    ej: np.ndarray      # int32 [m]
    w: np.ndarray       # f64 [m]
    u: np.ndarray       # f64 [m,3]

    @property
    def m(self):
        return int(self.ei.shape[0])


def collide(pos, radius, method: str = "auto", area: str = "overlap") -> Graph:
    """Collision graph (Section 2, Steps 1-2), canonical order.  w is the
    overlap (area="overlap") or the Hertz contact area pi R* overlap
    (area="hertz", the paper's benchmark cells, Section 5.1)."""
    pos = _c(pos, np.float64).reshape(-1, 3)
    radius = _c(radius, np.float64).reshape(-1)
    n = pos.shape[0]
    if method == "auto":
        method = "brute" if n <= 3000 else "cells"
    fn = lib().orc_collide_brute if method == "brute" else lib().orc_collide_cells
    st = C.c_int(0)
    gp = fn(C.c_int64(n), _f64(pos), _f64(radius), C.byref(st))
    if not gp:
        raise OracleError(st.value, "collide")
    g = gp.contents
    m = g.m

    def arr(ptr, cnt, dt):
        if cnt == 0:
            return np.zeros(0, dtype=dt)
        return np.ctypeslib.as_array(ptr, shape=(cnt,)).copy()

    out = Graph(n, arr(g.rowptr, n + 1, np.int32), arr(g.col, 2 * m, np.int32),
                arr(g.ei, m, np.int32), arr(g.ej, m, np.int32), arr(g.w, m, np.float64),
                arr(g.u, 3 * m, np.float64).reshape(m, 3))
    lib().orc_graph_free(gp)
    if area == "hertz":
        if m > 0:
            lib().orc_hertz_area(C.c_int64(m), _i32(out.ei), _i32(out.ej), _f64(radius), _f64(out.w))
    elif area != "overlap":
        raise ValueError(f"unknown contact area model {area!r}")
    return out


@dataclass
class BSR:
    n: int
    rowptr: np.ndarray  # int32 [n+1]
    bcol: np.ndarray    # int32 [nnzb]
    val: np.ndarray     # f64 [nnzb,3,3]

    def dense(self):
        n = self.n
        A = np.zeros((3 * n, 3 * n))
        for i in range(n):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                j = self.bcol[k]
                A[3 * i:3 * i + 3, 3 * j:3 * j + 3] = self.val[k]
        return A


def friction_block(w, u, g_par=G_PAR, g_perp=G_PERP):
    W = np.zeros(9)
    lib().orc_friction_block(C.c_double(w), _f64(_c(u, np.float64)), C.c_double(g_par),
                             C.c_double(g_perp), _f64(W))
    return W.reshape(3, 3)


def assemble(g: Graph, g_par=G_PAR, g_perp=G_PERP, g_med=G_MED) -> BSR:
    """Gamma as the block Laplacian of the collision graph (eq. cell_cell_friction, Def. Block Laplacian)."""
    n, m = g.n, g.m
    rowptr = np.zeros(n + 1, np.int32)
    bcol = np.zeros(n + 2 * m, np.int32)
    val = np.zeros((n + 2 * m) * 9, np.float64)
    st = lib().orc_assemble(C.c_int64(n), C.c_int64(m), _i32(g.rowptr), _i32(g.col), _i32(g.ei),
                            _i32(g.ej), _f64(g.w), _f64(_c(g.u, np.float64)), C.c_double(g_par),
                            C.c_double(g_perp), C.c_double(g_med), _i32(rowptr), _i32(bcol), _f64(val))
    if st != OK:
        raise OracleError(st, "assemble")
    return BSR(n, rowptr, bcol, val.reshape(-1, 3, 3))


def spmv(A: BSR, x):
    x = _c(x, np.float64).reshape(-1)
    y = np.zeros(3 * A.n)
    lib().orc_spmv(C.c_int64(A.n), _i32(A.rowptr), _i32(A.bcol), _f64(_c(A.val, np.float64)), _f64(x), _f64(y))
    return y.reshape(-1, 3)


def prim(g: Graph):
    """Prim's maximum spanning forest: (tree edges in Prim order, visit order)."""
    te = np.zeros(max(g.n, 1), np.int32)
    vis = np.zeros(max(g.n, 1), np.int32)
    nt = lib().orc_prim(C.c_int64(g.n), C.c_int64(g.m), _i32(g.ei), _i32(g.ej), _f64(g.w), _i32(te), _i32(vis))
    if nt < 0:
        raise OracleError(nt, "prim")
    return te[:nt].copy(), vis[:g.n].copy()


def kruskal(g: Graph):
    te = np.zeros(max(g.n, 1), np.int32)
    nt = lib().orc_kruskal(C.c_int64(g.n), C.c_int64(g.m), _i32(g.ei), _i32(g.ej), _f64(g.w), _i32(te))
    if nt < 0:
        raise OracleError(nt, "kruskal")
    return te[:nt].copy()


@dataclass
class Tree:
    n: int
    tree_edge: np.ndarray   # int32 [n-c], sorted ascending
    parent: np.ndarray      # int32 [n], -1 at roots
    pedge: np.ndarray       # int32 [n], edge to parent, -1 at roots
    depth: np.ndarray       # int32 [n]
    order: np.ndarray       # int32 [n], decreasing depth (elimination order of Alg. 2)
    child_ptr: np.ndarray   # int32 [n+1]
    child: np.ndarray       # int32 [n-c], ascending per parent


def build_tree(g: Graph, method: str = "prim") -> Tree:
    te = prim(g)[0] if method == "prim" else kruskal(g)
    te = np.sort(te).astype(np.int32)
    n = g.n
    parent = np.zeros(n, np.int32); pedge = np.zeros(n, np.int32); depth = np.zeros(n, np.int32)
    st = lib().orc_root_forest(C.c_int64(n), C.c_int64(te.shape[0]), _i32(te), _i32(g.ei), _i32(g.ej),
                               _i32(parent), _i32(pedge), _i32(depth))
    if st != OK:
        raise OracleError(st, "root_forest")
    order = np.zeros(n, np.int32); cptr = np.zeros(n + 1, np.int32); child = np.zeros(max(n, 1), np.int32)
    st = lib().orc_tree_order(C.c_int64(n), _i32(parent), _i32(depth), _i32(order), _i32(cptr), _i32(child))
    if st != OK:
        raise OracleError(st, "tree_order")
    return Tree(n, te, parent, pedge, depth, order, cptr, child[:int(cptr[n])].copy())


def forest_clusters(pos, radius, K, offsets=None):
    """Clusters of the local-MST forest (Section 6, Discussion): Z-order runs of
    K cells per instance."""
    pos = _c(pos, np.float64).reshape(-1, 3)
    radius = _c(radius, np.float64).reshape(-1)
    n = pos.shape[0]
    off = np.array([0, n], np.int64) if offsets is None else _c(offsets, np.int64)
    cl = np.zeros(max(n, 1), np.int32)
    st = lib().orc_forest_clusters(C.c_int64(n), _f64(pos), _f64(radius), C.c_int64(off.shape[0] - 1),
                                   _p(off, C.c_int64), C.c_int32(int(K)), _i32(cl))
    if st != OK:
        raise OracleError(st, "forest_clusters")
    return cl[:n].copy()


def build_forest(g: Graph, pos, radius, K, offsets=None):
    """The local-MST forest: Prim's maximum spanning forest of the graph
    without its edges between clusters, rooted as build_tree roots.  Returns
    (Tree, cluster of every cell)."""
    cl = forest_clusters(pos, radius, K, offsets)
    keep = np.nonzero(cl[g.ei] == cl[g.ej])[0].astype(np.int32) if g.m else np.zeros(0, np.int32)
    sub = Graph(g.n, g.rowptr, g.col, g.ei[keep], g.ej[keep], g.w[keep], g.u[keep])
    te_sub = prim(sub)[0]
    return tree_from_edges(g, keep[te_sub]), cl


def tree_from_edges(g: Graph, tree_edge) -> "Tree":
    """Root a forest given by its edge ids (each tree at its smallest vertex)."""
    te = np.sort(np.asarray(tree_edge)).astype(np.int32)
    n = g.n
    parent = np.zeros(n, np.int32); pedge = np.zeros(n, np.int32); depth = np.zeros(n, np.int32)
    st = lib().orc_root_forest(C.c_int64(n), C.c_int64(te.shape[0]), _i32(te), _i32(g.ei), _i32(g.ej),
                               _i32(parent), _i32(pedge), _i32(depth))
    if st != OK:
        raise OracleError(st, "root_forest")
    order = np.zeros(n, np.int32); cptr = np.zeros(n + 1, np.int32); child = np.zeros(max(n, 1), np.int32)
    st = lib().orc_tree_order(C.c_int64(n), _i32(parent), _i32(depth), _i32(order), _i32(cptr), _i32(child))
    if st != OK:
        raise OracleError(st, "tree_order")
    return Tree(n, te, parent, pedge, depth, order, cptr, child[:int(cptr[n])].copy())


@dataclass
class Factor:
    tree: Tree
    D: np.ndarray  # f64 [n,3,3] pivots
    L: np.ndarray  # f64 [n,3,3] L_{p(i),i}


def tree_factor(g: Graph, t: Tree, g_par=G_PAR, g_perp=G_PERP, g_med=G_MED) -> Factor:
    """TreeLDLT (Alg. 2) of the forest's block Laplacian P."""
    n = g.n
    D = np.zeros(9 * max(n, 1)); L = np.zeros(9 * max(n, 1))
    child = t.child if t.child.size else np.zeros(1, np.int32)
    st = lib().orc_tree_factor(C.c_int64(n), C.c_int64(t.tree_edge.shape[0]), _i32(t.tree_edge),
                               _i32(g.ei), _i32(g.ej), _f64(g.w), _f64(_c(g.u, np.float64)),
                               C.c_double(g_par), C.c_double(g_perp), C.c_double(g_med),
                               _i32(t.parent), _i32(t.pedge), _i32(t.order), _i32(t.child_ptr),
                               _i32(child), _f64(D), _f64(L))
    if st != OK:
        raise OracleError(st, "tree_factor")
    return Factor(t, D[:9 * n].reshape(n, 3, 3), L[:9 * n].reshape(n, 3, 3))


def tree_solve(f: Factor, b):
    """P^{-1} b by ForwardSolve, DiagSolve, BackwardSolve (Appendix B.1)."""
    t = f.tree
    b = _c(b, np.float64).reshape(-1)
    x = np.zeros(3 * t.n)
    child = t.child if t.child.size else np.zeros(1, np.int32)
    st = lib().orc_tree_solve(C.c_int64(t.n), _i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
                              _f64(_c(f.D, np.float64)), _f64(_c(f.L, np.float64)), _f64(b), _f64(x))
    if st != OK:
        raise OracleError(st, "tree_solve")
    return x.reshape(-1, 3)


def tree_solve_f32(f: Factor, b):
    """P^{-1} b by the FP32 tree solve of the refinement's inner solve
    (factor rounded to FP32, FP32 arithmetic), widened to FP64."""
    t = f.tree
    b = _c(b, np.float64).reshape(-1)
    x = np.zeros(3 * t.n)
    child = t.child if t.child.size else np.zeros(1, np.int32)
    st = lib().orc_tree_solve_f32(C.c_int64(t.n), _i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
                                  _f64(_c(f.D, np.float64)), _f64(_c(f.L, np.float64)), _f64(b), _f64(x))
    if st != OK:
        raise OracleError(st, "tree_solve_f32")
    return x.reshape(-1, 3)


def ir_inner(A: BSR, f: Factor, rhs, inner_tol=1e-5, max_iter=10_000, check=True):
    """One FP32 inner solve of the refinement: CG on Gamma d = rhs to relative
    inner_tol with FP32 product and sweeps.  Returns (d, iterations, status)."""
    t = f.tree
    rhs = _c(rhs, np.float64).reshape(-1)
    d = np.zeros(3 * A.n)
    it = np.zeros(1, np.int32)
    child = t.child if t.child.size else np.zeros(1, np.int32)
    st = lib().orc_ir_inner(C.c_int64(A.n), _i32(A.rowptr), _i32(A.bcol), _f64(_c(A.val, np.float64)),
                            _i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
                            _f64(_c(f.D, np.float64)), _f64(_c(f.L, np.float64)), _f64(rhs), _f64(d),
                            C.c_double(inner_tol), C.c_int(max_iter), _i32(it))
    if check and st != OK:
        raise OracleError(st, "ir_inner")
    return d.reshape(-1, 3), int(it[0]), int(st)


@dataclass
class SolveInfo:
    status: int
    iters: int
    relres_rec: float
    relres_true: float
    outer: int = 0


def pcg(A: BSR, F, prec: str = "tree", factor: Factor | None = None, x0=None, tol=1e-8,
        max_iter=10_000, fixed_iters=0, check=True):
    """Left-preconditioned CG (Section 1.1) with M = identity, block Jacobi or the tree."""
    n = A.n
    F = _c(F, np.float64).reshape(-1)
    x = np.zeros(3 * n) if x0 is None else _c(x0, np.float64).reshape(-1).copy()
    ii = np.zeros(1, np.int32); dd = np.zeros(2)
    z32 = np.zeros(1, np.int32); z64 = np.zeros(9)
    if prec == "tree":
        t = factor.tree
        child = t.child if t.child.size else z32
        tp = (_i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
              _f64(_c(factor.D, np.float64)), _f64(_c(factor.L, np.float64)))
    else:
        tp = (_i32(z32), _i32(z32), _i32(z32), _i32(z32), _f64(z64), _f64(z64))
    st = lib().orc_pcg(C.c_int64(n), _i32(A.rowptr), _i32(A.bcol), _f64(_c(A.val, np.float64)),
                       C.c_int(PREC[prec]), *tp, _f64(F), _f64(x), C.c_int(0 if x0 is None else 1),
                       C.c_double(tol), C.c_int(max_iter), C.c_int(fixed_iters), _i32(ii), _f64(dd))
    info = SolveInfo(int(st), int(ii[0]), float(dd[0]), float(dd[1]))
    if check and st != OK:
        raise OracleError(st, "pcg")
    return x.reshape(-1, 3), info


def pcg_gr(A: BSR, F, prec: str = "tree", factor: Factor | None = None, tol=1e-5, mu=1.0, max_iter=10_000,
           check=True):
    """PCG from zero stopped on an upper bound of the relative energy-norm
    error (Gauss-Radau with node mu <= lambda_min(P^-1 Gamma); orc_pcg_gr).
    Returns (x, info, hist) with info.relres the final error bound and
    hist[k] = (S_k, phi_k rho_k) for k = 0..iters."""
    n = A.n
    F = _c(F, np.float64).reshape(-1)
    x = np.zeros(3 * n)
    ii = np.zeros(1, np.int32); dd = np.zeros(2)
    hist = np.zeros(2 * (max_iter + 1))
    z32 = np.zeros(1, np.int32); z64 = np.zeros(9)
    if prec == "tree":
        t = factor.tree
        child = t.child if t.child.size else z32
        tp = (_i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
              _f64(_c(factor.D, np.float64)), _f64(_c(factor.L, np.float64)))
    else:
        tp = (_i32(z32), _i32(z32), _i32(z32), _i32(z32), _f64(z64), _f64(z64))
    st = lib().orc_pcg_gr(C.c_int64(n), _i32(A.rowptr), _i32(A.bcol), _f64(_c(A.val, np.float64)),
                          C.c_int(PREC[prec]), *tp, _f64(F), _f64(x), C.c_double(tol), C.c_double(mu),
                          C.c_int(max_iter), _i32(ii), _f64(dd), _f64(hist))
    info = SolveInfo(int(st), int(ii[0]), float(dd[0]), float(dd[1]))
    if check and st != OK:
        raise OracleError(st, "pcg_gr")
    k = int(ii[0])
    return x.reshape(-1, 3), info, hist[:2 * (k + 1)].reshape(-1, 2)


def ir_solve(A: BSR, F, factor: Factor, tol=1e-8, inner_tol=1e-5, max_outer=50, max_inner=10_000,
             check=True):
    """FP64 iterative refinement around an FP32 inner tree-PCG."""
    n = A.n
    t = factor.tree
    F = _c(F, np.float64).reshape(-1)
    x = np.zeros(3 * n)
    ii = np.zeros(2, np.int32); dd = np.zeros(1)
    child = t.child if t.child.size else np.zeros(1, np.int32)
    st = lib().orc_ir_solve(C.c_int64(n), _i32(A.rowptr), _i32(A.bcol), _f64(_c(A.val, np.float64)),
                            _i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
                            _f64(_c(factor.D, np.float64)), _f64(_c(factor.L, np.float64)),
                            _f64(F), _f64(x), C.c_double(tol), C.c_double(inner_tol),
                            C.c_int(max_outer), C.c_int(max_inner), _i32(ii), _f64(dd))
    info = SolveInfo(int(st), int(ii[0]), float(dd[0]), float("nan"), int(ii[1]))
    if check and st != OK:
        raise OracleError(st, "ir_solve")
    return x.reshape(-1, 3), info


def augment(g: Graph, t: Tree, t_parts=None):
    """Vaidya's augmented MST (Section 3.1): the MST cut into pieces of about
    n / t_parts cells (t_parts = ceil(n^(1/4)) by default; orc_aug_pieces),
    plus, for every pair of pieces joined by a contact, the heaviest such
    contact (ties: the smaller edge id).  Returns (edge ids of the augmented
    tree ascending, head of every cell's piece, added edge ids ascending)."""
    n = g.n
    if t_parts is None:
        t_parts = max(1, int(np.ceil(n ** 0.25)))
    s = max(1, -(-n // t_parts))
    piece = np.zeros(max(n, 1), np.int32)
    child = t.child if t.child.size else np.zeros(1, np.int32)
    st = lib().orc_aug_pieces(C.c_int64(n), _i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
                              C.c_int32(s), _i32(piece))
    if st != OK:
        raise OracleError(st, "aug_pieces")
    piece = piece[:n].copy()
    added = np.zeros(max(g.m, 1), np.int32)
    if g.m:
        st = lib().orc_aug_edges(C.c_int64(g.m), _i32(g.ei), _i32(g.ej), _f64(g.w), _i32(piece), _i32(added))
        if st != OK:
            raise OracleError(st, "aug_edges")
    add = np.nonzero(added[:g.m])[0].astype(np.int32)
    aug = np.union1d(t.tree_edge, add).astype(np.int32)
    return aug, piece, np.setdiff1d(add, t.tree_edge).astype(np.int32)


def assemble_edges(g: Graph, edges, g_par=G_PAR, g_perp=G_PERP, g_med=G_MED) -> BSR:
    """The block Laplacian (plus g_med I) of the subgraph with the given edge
    ids: assembly of the collision graph restricted to those contacts."""
    edges = np.asarray(edges, dtype=np.int32)
    ei, ej = g.ei[edges], g.ej[edges]
    n = g.n
    deg = np.bincount(np.concatenate([ei, ej]), minlength=n) if edges.size else np.zeros(n, np.int64)
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    rows = np.concatenate([ei, ej]); cols = np.concatenate([ej, ei])
    order = np.lexsort((cols, rows))
    sub = Graph(n, rowptr, cols[order].astype(np.int32), ei, ej, g.w[edges], g.u[edges])
    return assemble(sub, g_par, g_perp, g_med)


def fcg(A: BSR, Paug: BSR, f: Factor, F, tol=1e-8, inner_tol=0.1, max_iter=10_000, max_inner=10_000, x0=None,
        check=True):
    """Flexible CG on Gamma x = F whose preconditioner is tree-PCG on the
    augmented MST's Laplacian to relative residual inner_tol.  Returns
    (x, SolveInfo with iters = outer iterations, outer = inner iterations in all)."""
    n = A.n
    t = f.tree
    F = _c(F, np.float64).reshape(-1)
    x = np.zeros(3 * n) if x0 is None else _c(x0, np.float64).reshape(-1).copy()
    ii = np.zeros(2, np.int32); dd = np.zeros(2)
    child = t.child if t.child.size else np.zeros(1, np.int32)
    st = lib().orc_fcg(C.c_int64(n), _i32(A.rowptr), _i32(A.bcol), _f64(_c(A.val, np.float64)),
                       _i32(Paug.rowptr), _i32(Paug.bcol), _f64(_c(Paug.val, np.float64)),
                       _i32(t.parent), _i32(t.order), _i32(t.child_ptr), _i32(child),
                       _f64(_c(f.D, np.float64)), _f64(_c(f.L, np.float64)), _f64(F), _f64(x),
                       C.c_int(0 if x0 is None else 1), C.c_double(tol), C.c_double(inner_tol),
                       C.c_int(max_iter), C.c_int(max_inner), _i32(ii), _f64(dd))
    info = SolveInfo(int(st), int(ii[0]), float(dd[0]), float(dd[1]), int(ii[1]))
    if check and st != OK:
        raise OracleError(st, "fcg")
    return x.reshape(-1, 3), info


def forces(g: Graph, noise, k_rep=5.0):
    n = g.n
    noise = _c(noise, np.float64).reshape(-1)
    F = np.zeros(3 * n)
    lib().orc_forces(C.c_int64(n), _i32(g.rowptr), _i32(g.col), _i32(g.ei), _i32(g.ej), _f64(g.w),
                     _f64(_c(g.u, np.float64)), C.c_double(k_rep), _f64(noise), _f64(F))
    return F.reshape(-1, 3)


def euler(pos, v, dt):
    pos = _c(pos, np.float64).reshape(-1).copy()
    v = _c(v, np.float64).reshape(-1)
    lib().orc_euler(C.c_int64(pos.shape[0] // 3), C.c_double(dt), _f64(v), _f64(pos))
    return pos.reshape(-1, 3)


def solve_pipeline(pos, radius, F, prec="tree", tol=1e-8, max_iter=10_000, fixed_iters=0, x0=None,
                   g_par=G_PAR, g_perp=G_PERP, g_med=G_MED, check=True):
    """collide -> assemble -> Prim -> root -> TreeLDLT -> PCG, all in the oracle."""
    g = collide(pos, radius)
    A = assemble(g, g_par, g_perp, g_med)
    f = None
    t = None
    if prec == "tree":
        t = build_tree(g)
        f = tree_factor(g, t, g_par, g_perp, g_med)
    x, info = pcg(A, F, prec, f, x0=x0, tol=tol, max_iter=max_iter, fixed_iters=fixed_iters, check=check)
    return {"graph": g, "A": A, "tree": t, "factor": f, "x": x, "info": info}
