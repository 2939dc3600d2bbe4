"""ctypes binding of libsgp (include/sgp.h), same names as the C ABI.

Argument marshalling only: tensors are checked (CUDA/HIP device, dtype,
contiguity, shape), their device pointers and torch's current stream are
handed to the library, and status codes become SgpError.  torch provides the
device memory and the stream; every step of the method runs in libsgp.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsgp.so")

OK, EINVAL, ENOMEM, EHIP, ECAPACITY, ENOTSPD, ENOCONV, EBREAKDOWN, ENONFINITE, ESTALE = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
SCHED_LEVEL, SCHED_CONTRACT = 0, 1
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ECAPACITY", -5: "ENOTSPD",
           -6: "ENOCONV", -7: "EBREAKDOWN", -8: "ENONFINITE", -9: "ESTALE"}

_lib = None


class SgpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("fixed_iters", C.c_int32),
                ("use_x0", C.c_int32), ("precision", C.c_int32), ("inner_rtol", C.c_double),
                ("max_outer", C.c_int32), ("check_every", C.c_int32), ("stop", C.c_int32),
                ("reserved", C.c_int32), ("mu", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer_iters", C.c_int32),
                ("inner_iters", C.c_int32), ("relres_rec", C.c_double), ("relres_true", C.c_double),
                ("err_bound", C.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters, "outer_iters": self.outer_iters,
                "inner_iters": self.inner_iters, "relres_rec": self.relres_rec, "relres_true": self.relres_true,
                "err_bound": self.err_bound}


STOP = {"residual": 0, "error": 1}


_vp, _i64, _i32, _dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
_SIGS = {
    "sgp_create": (C.c_int, [C.POINTER(_vp), _vp]),
    "sgp_destroy": (None, [_vp]),
    "sgp_last_error": (C.c_char_p, [_vp]),
    "sgp_set_stream": (C.c_int, [_vp, _vp]),
    "sgp_graph_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "sgp_graph_free": (None, [_vp]),
    "sgp_collide": (C.c_int, [_vp, _i64, _vp, _vp, _i32, _vp]),
    "sgp_collide_batched": (C.c_int, [_vp, _i64, C.POINTER(_i64), _vp, _vp, _i32, _vp]),
    "sgp_graph_size": (C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i64)]),
    "sgp_graph_export": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sgp_bsr_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "sgp_bsr_free": (None, [_vp]),
    "sgp_assemble_gamma": (C.c_int, [_vp, _vp, _dbl, _dbl, _dbl, _vp]),
    "sgp_bsr_size": (C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i64)]),
    "sgp_bsr_export": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "sgp_spmv": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sgp_tree_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "sgp_tree_free": (None, [_vp]),
    "sgp_build_tree": (C.c_int, [_vp, _vp, _vp]),
    "sgp_tree_size": (C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32)]),
    "sgp_tree_export": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "sgp_prec_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "sgp_prec_free": (None, [_vp]),
    "sgp_factor_tree": (C.c_int, [_vp, _vp, _vp, _dbl, _dbl, _dbl, _i32, _vp]),
    "sgp_make_jacobi": (C.c_int, [_vp, _vp, _vp]),
    "sgp_prec_steps": (C.c_int, [_vp, C.POINTER(_i32)]),
    "sgp_prec_apply": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sgp_prec_apply_noalloc": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sgp_set_contact_model": (C.c_int, [_vp, _i32]),
    "sgp_build_forest": (C.c_int, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "sgp_factor_augmented": (C.c_int, [_vp, _vp, _vp, _dbl, _dbl, _dbl, _i32, _i32, _dbl, _vp]),
    "sgp_prec_augmented": (C.c_int, [_vp, _vp, C.POINTER(_i64), C.POINTER(_i64), _vp, _vp]),
    "sgp_tree_clusters": (C.c_int, [_vp, _vp, _vp, C.POINTER(_i64)]),
    "sgp_step_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "sgp_step_free": (None, [_vp]),
    "sgp_step_record_batched": (C.c_int, [_vp, _vp, _i64, C.POINTER(_i64), _vp, _vp, _i32, _dbl, _dbl, _dbl, _i32,
                                          _i32, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "sgp_step_replay": (C.c_int, [_vp, _vp, C.POINTER(SolveInfo)]),
    "sgp_step_size": (C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i64)]),
    "sgp_pcg_solve": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "sgp_pcg_solve_batched": (C.c_int, [_vp, _vp, _vp, _i64, C.POINTER(_i64), _vp, _vp,
                                        C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "sgp_forces": (C.c_int, [_vp, _vp, _dbl, _vp, _vp]),
    "sgp_euler": (C.c_int, [_vp, _i64, _dbl, _vp, _vp]),
    "sgp_phase_times": (C.c_int, [_vp, C.POINTER(_dbl)]),
    "sgp_tune": (C.c_int, [_vp, C.c_char_p, _i32]),
    "sgp_prec_info": (C.c_int, [_vp, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32), _vp]),
    "sgp_tune_get": (C.c_int, [_vp, C.c_char_p, C.POINTER(_i32)]),
    "sgp_kernel_timing": (C.c_int, [_vp, _i32]),
    "sgp_residual_norm": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(_dbl)]),
    "sgp_mpnn_param_count": (C.c_int, [C.POINTER(_i64)]),
    "sgp_mpnn_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "sgp_mpnn_free": (None, [_vp]),
    "sgp_mpnn_set_params": (C.c_int, [_vp, _vp, _vp, _dbl, _dbl, _dbl]),
    "sgp_mpnn_get_params": (C.c_int, [_vp, _vp, _vp]),
    "sgp_mpnn_forward": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "sgp_mpnn_grad": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_dbl)]),
    "sgp_mpnn_train_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _dbl, C.POINTER(_dbl)]),
    "sgp_mpnn_warm_start": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_i32), C.POINTER(_dbl),
                                      C.POINTER(_dbl)]),
    "sgp_kernel_stats": (C.c_int, [_vp, C.POINTER(_dbl), C.POINTER(_i64)]),
}


def lib():
    """Load libsgp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsgp.so not found at {LIB_PATH}: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t: torch.Tensor | None, dtype=None, what="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise SgpError(EINVAL, f"{what} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise SgpError(EINVAL, f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise SgpError(EINVAL, f"{what} must be contiguous")
    return C.c_void_p(t.data_ptr())


class _Handle:
    _free = None

    def __init__(self, ctx, create):
        self.ctx = ctx
        self.h = C.c_void_p()
        ctx._check(getattr(lib(), create)(ctx.h, C.byref(self.h)), create)

    def __del__(self):
        try:
            if self.h and self.h.value and _lib is not None:
                getattr(_lib, self._free)(self.h)
                self.h = C.c_void_p()
        except Exception:
            pass


class Graph(_Handle):
    _free = "sgp_graph_free"

    def __init__(self, ctx):
        super().__init__(ctx, "sgp_graph_create")
        self.offsets = None

    def size(self):
        n, m = C.c_int64(), C.c_int64()
        lib().sgp_graph_size(self.h, C.byref(n), C.byref(m))
        return n.value, m.value


class Bsr(_Handle):
    _free = "sgp_bsr_free"

    def __init__(self, ctx):
        super().__init__(ctx, "sgp_bsr_create")

    def size(self):
        n, nnzb = C.c_int64(), C.c_int64()
        lib().sgp_bsr_size(self.h, C.byref(n), C.byref(nnzb))
        return n.value, nnzb.value


class Tree(_Handle):
    _free = "sgp_tree_free"

    def __init__(self, ctx):
        super().__init__(ctx, "sgp_tree_create")

    def size(self):
        nt, nr, md = C.c_int64(), C.c_int64(), C.c_int32()
        lib().sgp_tree_size(self.h, C.byref(nt), C.byref(nr), C.byref(md))
        return nt.value, nr.value, md.value


class Prec(_Handle):
    _free = "sgp_prec_free"

    def __init__(self, ctx):
        super().__init__(ctx, "sgp_prec_create")

    def steps(self):
        s = C.c_int32()
        lib().sgp_prec_steps(self.h, C.byref(s))
        return s.value

    def info(self):
        """{"steps", "tail_step", "light_steps", "step_sizes"} of the schedule."""
        s, t, lt = C.c_int32(), C.c_int32(), C.c_int32()
        lib().sgp_prec_info(self.h, C.byref(s), C.byref(t), C.byref(lt), None)
        sizes = (C.c_int32 * max(s.value, 1))()
        lib().sgp_prec_info(self.h, C.byref(s), C.byref(t), C.byref(lt), sizes)
        return {"steps": s.value, "tail_step": t.value, "light_steps": lt.value,
                "step_sizes": [sizes[k] for k in range(s.value)]}


class Step(_Handle):
    """A batched step recorded once and replayed as one hipGraph (sgp_step_*).
    Keeps the tensors it was recorded with alive."""
    _free = "sgp_step_free"

    def __init__(self, ctx):
        super().__init__(ctx, "sgp_step_create")
        self.keep = None

    def size(self):
        v, b = C.c_int64(), C.c_int64()
        lib().sgp_step_size(self.h, C.byref(v), C.byref(b))
        return v.value, b.value

    def record_batched(self, offsets, pos, radius, F, v, prec="tree", g_par=1.0, g_perp=0.1, g_med=1e-3,
                       schedule="contract", max_deg=32, rtol=1e-8, max_iter=10000, use_x0=False, check_every=0):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        k = off.shape[0] - 1
        o = self.ctx._opts(rtol, max_iter, 0, use_x0, "f64", 1e-5, 50, check_every)
        infos = (SolveInfo * k)()
        code = {"none": 0, "jacobi": 1, "tree": 2}[prec]
        sch = {"level": SCHED_LEVEL, "contract": SCHED_CONTRACT}[schedule]
        self.keep = (pos, radius, F, v)
        self.ctx._check(lib().sgp_step_record_batched(
            self.ctx.h, self.h, k, off.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(pos, torch.float64, "pos"),
            _ptr(radius, torch.float64, "radius"), max_deg, g_par, g_perp, g_med, code, sch,
            _ptr(F, torch.float64, "F"), _ptr(v, torch.float64, "v"), C.byref(o), infos), "sgp_step_record_batched")
        self.n_inst = k
        return [infos[i].as_dict() for i in range(k)]

    def replay(self, check=True):
        infos = (SolveInfo * self.n_inst)()
        st = lib().sgp_step_replay(self.ctx.h, self.h, infos)
        if check:
            self.ctx._check(st, "sgp_step_replay")
        return st, [infos[i].as_dict() for i in range(self.n_inst)]


class Mpnn(_Handle):
    """Learned warm start network (parameters live on the device)."""
    _free = "sgp_mpnn_free"

    def __init__(self, ctx):
        super().__init__(ctx, "sgp_mpnn_create")

    @staticmethod
    def param_count():
        c = C.c_int64()
        lib().sgp_mpnn_param_count(C.byref(c))
        return c.value

    def set_params(self, theta, sF, sV, sW):
        t = torch.as_tensor(theta, dtype=torch.float32).to(self.ctx.dev()).contiguous()
        if t.numel() != self.param_count():
            raise SgpError(EINVAL, "wrong parameter count")
        self.ctx._check(lib().sgp_mpnn_set_params(self.ctx.h, self.h, _ptr(t), sF, sV, sW), "sgp_mpnn_set_params")

    def get_params(self):
        t = torch.empty(self.param_count(), dtype=torch.float32, device=self.ctx.dev())
        self.ctx._check(lib().sgp_mpnn_get_params(self.ctx.h, self.h, _ptr(t)), "sgp_mpnn_get_params")
        return t

    def forward(self, g, F, vprev, out=None):
        out = torch.empty_like(F) if out is None else out
        self.ctx._check(lib().sgp_mpnn_forward(self.ctx.h, self.h, g.h, _ptr(F, torch.float64, "F"),
                                               _ptr(vprev, torch.float64, "vprev"), _ptr(out, torch.float64, "vhat")),
                        "sgp_mpnn_forward")
        return out

    def grad(self, g, F, vprev, v, A: "Bsr | None" = None):
        """Loss and gradient; energy loss when Gamma (A) is given, else MSE."""
        gr = torch.empty(self.param_count(), dtype=torch.float32, device=self.ctx.dev())
        loss = C.c_double()
        self.ctx._check(lib().sgp_mpnn_grad(self.ctx.h, self.h, g.h, A.h if A is not None else None,
                                            _ptr(F, torch.float64, "F"), _ptr(vprev, torch.float64, "vprev"),
                                            _ptr(v, torch.float64, "v"), _ptr(gr), C.byref(loss)), "sgp_mpnn_grad")
        return loss.value, gr

    def train_step(self, g, F, vprev, v, lr, A: "Bsr | None" = None):
        loss = C.c_double()
        self.ctx._check(lib().sgp_mpnn_train_step(self.ctx.h, self.h, g.h, A.h if A is not None else None,
                                                  _ptr(F, torch.float64, "F"), _ptr(vprev, torch.float64, "vprev"),
                                                  _ptr(v, torch.float64, "v"), lr, C.byref(loss)),
                        "sgp_mpnn_train_step")
        return loss.value

    def warm_start(self, g, A, F, vprev, x0=None):
        """Initial guess: v_prev, the network's v_hat or zero, whichever has the
        lowest energy under Gamma.  Returns (x0, {"used_net", "used_zero",
        "energy_net", "energy_prev"})."""
        x0 = torch.empty_like(vprev) if x0 is None else x0
        used = C.c_int32()
        en, ep = C.c_double(), C.c_double()
        self.ctx._check(lib().sgp_mpnn_warm_start(self.ctx.h, self.h, g.h, A.h, _ptr(F, torch.float64, "F"),
                                                  _ptr(vprev, torch.float64, "vprev"), _ptr(x0, torch.float64, "x0"),
                                                  C.byref(used), C.byref(en), C.byref(ep)), "sgp_mpnn_warm_start")
        return x0, {"used_net": used.value == 1, "used_zero": used.value == 2, "energy_net": en.value,
                    "energy_prev": ep.value}


class Context:
    """One libsgp context on the current device, ordered on a torch stream."""

    def __init__(self, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libsgp needs a GPU (torch.cuda.is_available() is False)")
        self.stream = stream or torch.cuda.current_stream()
        self.h = C.c_void_p()
        st = lib().sgp_create(C.byref(self.h), C.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise SgpError(st, "sgp_create failed")

    def close(self):
        if self.h and self.h.value:
            lib().sgp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, status, what):
        if status != OK:
            msg = lib().sgp_last_error(self.h).decode() if self.h else ""
            raise SgpError(status, f"{what}: {msg}")

    def dev(self):
        return torch.device("cuda", torch.cuda.current_device())

    # ---------------------------------------------------------------- Steps 1-2
    def set_contact_model(self, model: str):
        """What later collides store as w: "overlap" (default) or "hertz"."""
        code = {"overlap": 0, "hertz": 1}[model]
        self._check(lib().sgp_set_contact_model(self.h, code), "sgp_set_contact_model")

    def collide(self, pos, radius, max_deg=32, g: Graph | None = None) -> Graph:
        n = pos.shape[0]
        if pos.shape != (n, 3) or radius.shape != (n,):
            raise SgpError(EINVAL, "pos must be [n,3] and radius [n]")
        g = g or Graph(self)
        self._check(lib().sgp_collide(self.h, n, _ptr(pos, torch.float64, "pos"),
                                      _ptr(radius, torch.float64, "radius"), max_deg, g.h), "sgp_collide")
        g.offsets = None
        return g

    def collide_batched(self, offsets, pos, radius, max_deg=32, g: Graph | None = None) -> Graph:
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        k = off.shape[0] - 1
        if pos.shape != (int(off[-1]), 3) or radius.shape != (int(off[-1]),):
            raise SgpError(EINVAL, "pos/radius do not match offsets")
        g = g or Graph(self)
        self._check(lib().sgp_collide_batched(self.h, k, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                              _ptr(pos, torch.float64, "pos"),
                                              _ptr(radius, torch.float64, "radius"), max_deg, g.h),
                    "sgp_collide_batched")
        g.offsets = off
        return g

    def graph_export(self, g: Graph):
        n, m = g.size()
        d = self.dev()
        out = {"rowptr": torch.empty(n + 1, dtype=torch.int32, device=d),
               "col": torch.empty(2 * m, dtype=torch.int32, device=d),
               "ei": torch.empty(m, dtype=torch.int32, device=d),
               "ej": torch.empty(m, dtype=torch.int32, device=d),
               "w": torch.empty(m, dtype=torch.float64, device=d),
               "u": torch.empty((m, 3), dtype=torch.float64, device=d)}
        self._check(lib().sgp_graph_export(self.h, g.h, *[_ptr(out[k]) for k in
                                                            ("rowptr", "col", "ei", "ej", "w", "u")]),
                    "sgp_graph_export")
        return out

    # ---------------------------------------------------------------- Step 3
    def assemble_gamma(self, g: Graph, g_par=1.0, g_perp=0.1, g_med=1e-3, A: Bsr | None = None) -> Bsr:
        A = A or Bsr(self)
        self._check(lib().sgp_assemble_gamma(self.h, g.h, g_par, g_perp, g_med, A.h), "sgp_assemble_gamma")
        return A

    def bsr_export(self, A: Bsr):
        n, nnzb = A.size()
        d = self.dev()
        out = {"rowptr": torch.empty(n + 1, dtype=torch.int32, device=d),
               "bcol": torch.empty(nnzb, dtype=torch.int32, device=d),
               "val": torch.empty((nnzb, 3, 3), dtype=torch.float64, device=d)}
        self._check(lib().sgp_bsr_export(self.h, A.h, _ptr(out["rowptr"]), _ptr(out["bcol"]), _ptr(out["val"])),
                    "sgp_bsr_export")
        return out

    def spmv(self, A: Bsr, x, y=None):
        y = torch.empty_like(x) if y is None else y
        self._check(lib().sgp_spmv(self.h, A.h, _ptr(x, torch.float64, "x"), _ptr(y, torch.float64, "y")),
                    "sgp_spmv")
        return y

    # ---------------------------------------------------------------- Section 3.1
    def build_tree(self, g: Graph, T: Tree | None = None) -> Tree:
        T = T or Tree(self)
        self._check(lib().sgp_build_tree(self.h, g.h, T.h), "sgp_build_tree")
        return T

    def build_forest(self, g: Graph, pos, radius, cluster_size=512, T: Tree | None = None) -> Tree:
        """Local maximum spanning forest: one per Z-order cluster of cluster_size cells."""
        T = T or Tree(self)
        self._check(lib().sgp_build_forest(self.h, g.h, _ptr(pos, torch.float64, "pos"),
                                           _ptr(radius, torch.float64, "radius"), cluster_size, T.h),
                    "sgp_build_forest")
        return T

    def tree_clusters(self, T: Tree, n: int):
        """(cluster of every cell as a device int32 tensor, number of clusters)."""
        nc = C.c_int64()
        out = torch.empty(n, dtype=torch.int32, device=self.dev())
        self._check(lib().sgp_tree_clusters(self.h, T.h, _ptr(out, torch.int32, "cluster"), C.byref(nc)),
                    "sgp_tree_clusters")
        return out, nc.value

    def tree_export(self, T: Tree, n: int):
        nt, _, _ = T.size()
        d = self.dev()
        out = {"tree_edge": torch.empty(nt, dtype=torch.int32, device=d),
               "parent": torch.empty(n, dtype=torch.int32, device=d),
               "depth": torch.empty(n, dtype=torch.int32, device=d)}
        self._check(lib().sgp_tree_export(self.h, T.h, _ptr(out["tree_edge"]), _ptr(out["parent"]),
                                          _ptr(out["depth"])), "sgp_tree_export")
        return out

    # ---------------------------------------------------------------- Section 3.3
    def factor_tree(self, g: Graph, T: Tree, g_par=1.0, g_perp=0.1, g_med=1e-3, schedule="contract",
                    M: Prec | None = None) -> Prec:
        M = M or Prec(self)
        sch = {"level": SCHED_LEVEL, "contract": SCHED_CONTRACT}[schedule] if isinstance(schedule, str) else schedule
        self._check(lib().sgp_factor_tree(self.h, g.h, T.h, g_par, g_perp, g_med, sch, M.h), "sgp_factor_tree")
        return M

    def factor_augmented(self, g: Graph, T: Tree, g_par=1.0, g_perp=0.1, g_med=1e-3, schedule="contract",
                         parts=0, inner_rtol=0.1, M: Prec | None = None) -> Prec:
        """Vaidya's augmented tree with the nested (flexible CG) solve."""
        M = M or Prec(self)
        sch = {"level": SCHED_LEVEL, "contract": SCHED_CONTRACT}[schedule]
        self._check(lib().sgp_factor_augmented(self.h, g.h, T.h, g_par, g_perp, g_med, sch, parts, inner_rtol, M.h),
                    "sgp_factor_augmented")
        return M

    def prec_augmented(self, M: Prec, n: int):
        """(pieces, added, head of every cell's piece, added edge ids) of an augmented tree."""
        npc, nad = C.c_int64(), C.c_int64()
        self._check(lib().sgp_prec_augmented(self.h, M.h, C.byref(npc), C.byref(nad), None, None),
                    "sgp_prec_augmented")
        piece = torch.empty(n, dtype=torch.int32, device=self.dev())
        added = torch.empty(max(nad.value, 1), dtype=torch.int32, device=self.dev())
        self._check(lib().sgp_prec_augmented(self.h, M.h, None, None, _ptr(piece, torch.int32, "piece"),
                                             _ptr(added, torch.int32, "added")), "sgp_prec_augmented")
        return npc.value, nad.value, piece, added[:nad.value]

    def make_jacobi(self, A: Bsr, M: Prec | None = None) -> Prec:
        M = M or Prec(self)
        self._check(lib().sgp_make_jacobi(self.h, A.h, M.h), "sgp_make_jacobi")
        return M

    def prec_apply(self, M: Prec, r, z=None):
        z = torch.empty_like(r) if z is None else z
        self._check(lib().sgp_prec_apply(self.h, M.h, _ptr(r, torch.float64, "r"), _ptr(z, torch.float64, "z")),
                    "sgp_prec_apply")
        return z

    def prec_apply_noalloc(self, M: Prec, r, z):
        """z = M^{-1} r through the entry point that allocates nothing (static
        device scratch; at most 2^20 cells); z must be given."""
        self._check(lib().sgp_prec_apply_noalloc(self.h, M.h, _ptr(r, torch.float64, "r"),
                                                 _ptr(z, torch.float64, "z")), "sgp_prec_apply_noalloc")
        return z

    # ---------------------------------------------------------------- Section 1.1
    @staticmethod
    def _opts(rtol, max_iter, fixed_iters, use_x0, precision, inner_rtol, max_outer, check_every, stop="residual",
              mu=0.0):
        return SolveOpts(rtol, max_iter, fixed_iters, 1 if use_x0 else 0,
                         {"f64": 0, "f32ir": 1}[precision], inner_rtol, max_outer, check_every, STOP[stop], 0, mu)

    def pcg_solve(self, A: Bsr, M: Prec | None, F, v=None, rtol=1e-8, max_iter=10000, fixed_iters=0,
                  use_x0=False, precision="f64", inner_rtol=1e-5, max_outer=50, check_every=0, check=True,
                  stop="residual", mu=0.0):
        """stop="error": rtol bounds the relative energy-norm error (Gauss-Radau
        with node mu; 0 = the default of sgp_solve_opts.mu)."""
        if v is None:
            v = torch.zeros_like(F)
            use_x0 = False
        o = self._opts(rtol, max_iter, fixed_iters, use_x0, precision, inner_rtol, max_outer, check_every, stop, mu)
        info = SolveInfo()
        st = lib().sgp_pcg_solve(self.h, A.h, M.h if M is not None else None, _ptr(F, torch.float64, "F"),
                                 _ptr(v, torch.float64, "v"), C.byref(o), C.byref(info))
        if check and st not in (OK,):
            self._check(st, "sgp_pcg_solve")
        return v, info.as_dict()

    def pcg_solve_batched(self, A: Bsr, M: Prec | None, offsets, F, v=None, rtol=1e-8, max_iter=10000,
                          fixed_iters=0, use_x0=False, check_every=0, check=True, stop="residual", mu=0.0):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        k = off.shape[0] - 1
        if v is None:
            v = torch.zeros_like(F)
            use_x0 = False
        o = self._opts(rtol, max_iter, fixed_iters, use_x0, "f64", 1e-5, 50, check_every, stop, mu)
        infos = (SolveInfo * k)()
        st = lib().sgp_pcg_solve_batched(self.h, A.h, M.h if M is not None else None, k,
                                         off.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(F, torch.float64, "F"),
                                         _ptr(v, torch.float64, "v"), C.byref(o), infos)
        if check and st != OK:
            self._check(st, "sgp_pcg_solve_batched")
        return v, [infos[i].as_dict() for i in range(k)]

    def residual_norm(self, A: Bsr, F, x):
        r = C.c_double()
        self._check(lib().sgp_residual_norm(self.h, A.h, _ptr(F, torch.float64, "F"), _ptr(x, torch.float64, "x"),
                                            C.byref(r)), "sgp_residual_norm")
        return r.value

    # ---------------------------------------------------------------- dynamics
    def forces(self, g: Graph, noise, k_rep=5.0, F=None):
        F = torch.empty_like(noise) if F is None else F
        self._check(lib().sgp_forces(self.h, g.h, k_rep, _ptr(noise, torch.float64, "noise"),
                                     _ptr(F, torch.float64, "F")), "sgp_forces")
        return F

    def euler(self, pos, v, dt):
        self._check(lib().sgp_euler(self.h, pos.shape[0], dt, _ptr(v, torch.float64, "v"),
                                    _ptr(pos, torch.float64, "pos")), "sgp_euler")
        return pos

    def phase_times(self):
        a = (C.c_double * 5)()
        lib().sgp_phase_times(self.h, a)
        return dict(zip(("collide", "assemble", "build_tree", "factor", "solve"), list(a)))

    def kernel_timing(self, enable: bool):
        self._check(lib().sgp_kernel_timing(self.h, 1 if enable else 0), "sgp_kernel_timing")

    def kernel_stats(self):
        ms, cnt = C.c_double(), C.c_int64()
        self._check(lib().sgp_kernel_stats(self.h, C.byref(ms), C.byref(cnt)), "sgp_kernel_stats")
        return ms.value, cnt.value

    def tune(self, key: str, value: int):
        self._check(lib().sgp_tune(self.h, key.encode(), int(value)), "sgp_tune")

    def tune_get(self, key: str) -> int:
        v = C.c_int32()
        self._check(lib().sgp_tune_get(self.h, key.encode(), C.byref(v)), "sgp_tune_get")
        return v.value
