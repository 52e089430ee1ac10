"""ctypes binding of the C ABI in include/tufrg.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
CHANNELS = ("P", "C", "D")
IRREPS = ("A1", "B1", "B2", "A2", "E")

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENONFINITE", -5: "EUNSUPPORTED"}
FLOW_STATUS = {1: "diverged", 2: "reached_tmin", 3: "nonfinite", 4: "max_steps"}
SCHEMES = {"rk4": 0, "dopri5": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}
NO_CROSS = 1
AUTOTUNE = 2
LOOP_QUEUE = 4
NO_SYMMETRY = 8
NO_FUSE = 16
OMEGA_CUTOFF = 32
SYMMETRIC_STATE = 64
DENSE_PROJECTION = 128
NO_LOOP_REUSE = 256
REGULATORS = {"T": 0, "omega": OMEGA_CUTOFF}

# every entry point declared in include/tufrg.h
EXPORTS = ("tufrg_init", "tufrg_init_mesh", "tufrg_layout", "tufrg_geometry", "tufrg_bubbles", "tufrg_project",
           "tufrg_rhs", "tufrg_rhs_noalloc", "tufrg_flow", "tufrg_symmetry_defect", "tufrg_sync", "tufrg_flop_count", "tufrg_loop_kernel_time",
           "tufrg_kernel_times",
           "tufrg_mu_from_filling",
           "tufrg_harmonics", "tufrg_loop_harmonics", "tufrg_surrogate_dataset",
           "tufrg_surrogate_attach", "tufrg_surrogate_stats",
           "tufrg_mlp_create", "tufrg_mlp_nparams", "tufrg_mlp_get_params", "tufrg_mlp_set_params",
           "tufrg_mlp_forward", "tufrg_mlp_gradient", "tufrg_mlp_train", "tufrg_mlp_free",
           "tufrg_mlp_last_error", "tufrg_free", "tufrg_last_error")
NO_STATUS = ("tufrg_free", "tufrg_last_error", "tufrg_mlp_free", "tufrg_mlp_last_error")


class TufrgError(RuntimeError):
    pass


class _Point(C.Structure):
    _fields_ = [("t", C.c_double), ("tp", C.c_double), ("mu", C.c_double), ("U", C.c_double),
                ("Lq", C.c_int32), ("Lk", C.c_int32), ("shells", C.c_int32),
                ("reserved", C.c_int32)]


class _Mesh(C.Structure):
    _fields_ = [("nq", C.c_int32), ("qx", C.POINTER(C.c_double)), ("qy", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double))]


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("flags", C.c_uint32)]


class _FlowOpts(C.Structure):
    _fields_ = [("T0", C.c_double), ("Tmin", C.c_double), ("Xmax", C.c_double),
                ("scheme", C.c_int32), ("nsteps", C.c_int32), ("rtol", C.c_double),
                ("atol", C.c_double), ("h0", C.c_double), ("max_steps", C.c_int32),
                ("use_graph", C.c_int32)]


class _FlowResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("channel", C.c_int32), ("q_index", C.c_int32),
                ("irrep", C.c_int32), ("Tc", C.c_double), ("max_abs_X", C.c_double),
                ("max_abs_V", C.c_double), ("n_rhs", C.c_int64), ("n_steps", C.c_int64)]


_LIB = None


def library_path() -> str:
    return os.path.join(HERE, "_lib", "libtufrg.so")


def load_library():
    """Load the built native library; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise TufrgError(f"native library missing: {path} (run python -m paper_1604_06296_amd.build)")
    lib = C.CDLL(path)
    vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
    lib.tufrg_init.argtypes = [C.POINTER(_Point), i32, C.POINTER(_Options), vp, C.POINTER(vp)]
    lib.tufrg_init_mesh.argtypes = [C.POINTER(_Point), C.POINTER(_Mesh), i32, C.POINTER(_Options), vp,
                                    C.POINTER(vp)]
    lib.tufrg_layout.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                 C.POINTER(i64)]
    lib.tufrg_geometry.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                   C.POINTER(i32)]
    lib.tufrg_bubbles.argtypes = [vp, dp, vp]
    lib.tufrg_project.argtypes = [vp, vp, vp]
    lib.tufrg_rhs.argtypes = [vp, dp, vp, vp]
    lib.tufrg_rhs_noalloc.argtypes = [vp, dp, vp, vp]
    lib.tufrg_flow.argtypes = [vp, C.POINTER(_FlowOpts), vp, C.POINTER(_FlowResult)]
    lib.tufrg_sync.argtypes = [vp]
    lib.tufrg_symmetry_defect.argtypes = [vp, vp, dp]
    lib.tufrg_flop_count.argtypes = [vp, dp]
    lib.tufrg_loop_kernel_time.argtypes = [vp, dp, i32, dp, dp]
    lib.tufrg_kernel_times.argtypes = [vp, dp, vp, vp, i32, dp, dp]
    lib.tufrg_mu_from_filling.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, i32, dp]
    u64, f32 = C.c_uint64, C.c_float
    lib.tufrg_harmonics.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)]
    lib.tufrg_loop_harmonics.argtypes = [vp, dp, vp]
    lib.tufrg_surrogate_dataset.argtypes = [vp, dp, i64, u64, vp, vp, vp]
    lib.tufrg_surrogate_attach.argtypes = [vp, vp, vp, C.c_double, i32]
    lib.tufrg_surrogate_stats.argtypes = [vp, C.POINTER(i64)]
    lib.tufrg_mlp_create.argtypes = [C.POINTER(i32), i32, i32, u64, vp, C.POINTER(vp)]
    lib.tufrg_mlp_nparams.argtypes = [vp, C.POINTER(i64)]
    lib.tufrg_mlp_get_params.argtypes = [vp, vp]
    lib.tufrg_mlp_set_params.argtypes = [vp, vp]
    lib.tufrg_mlp_forward.argtypes = [vp, vp, vp, i64]
    lib.tufrg_mlp_gradient.argtypes = [vp, vp, vp, i64, vp, dp]
    lib.tufrg_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, f32, u64, dp]
    lib.tufrg_mlp_free.argtypes = [vp]
    lib.tufrg_mlp_free.restype = None
    lib.tufrg_mlp_last_error.argtypes = [vp]
    lib.tufrg_mlp_last_error.restype = C.c_char_p
    lib.tufrg_free.argtypes = [vp]
    lib.tufrg_free.restype = None
    lib.tufrg_last_error.argtypes = [vp]
    lib.tufrg_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in NO_STATUS:
            getattr(lib, name).restype = C.c_int
    _LIB = lib
    return lib


def _check(lib, ctx, status):
    if status != 0:
        msg = lib.tufrg_last_error(ctx).decode()
        raise TufrgError(f"{STATUS.get(status, status)}: {msg}")


def _check_mlp(lib, net, status):
    if status != 0:
        msg = lib.tufrg_mlp_last_error(net).decode()
        raise TufrgError(f"{STATUS.get(status, status)}: {msg}")


def _dev_array(x, dtype, numel=None, what="array"):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dtype and x.is_contiguous()):
        raise TufrgError(f"{what}: expected a contiguous {dtype} CUDA tensor")
    if numel is not None and x.numel() != numel:
        raise TufrgError(f"{what}: expected {numel} elements, got {x.numel()}")
    return C.c_void_p(x.data_ptr())


class MLP:
    """Surrogate network (tufrg_mlp_*): SiLU MLP trained with the library's kernels."""

    def __init__(self, widths: Sequence[int], max_rows: int = 65536, seed: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise TufrgError("a GPU is required (torch.cuda.is_available() is False)")
        self._torch = torch
        self.lib = load_library()
        self.widths = [int(w) for w in widths]
        self.max_rows = int(max_rows)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (C.c_int32 * len(self.widths))(*self.widths)
        handle = C.c_void_p()
        _check_mlp(self.lib, None, self.lib.tufrg_mlp_create(arr, len(self.widths), self.max_rows,
                                                             C.c_uint64(seed),
                                                             C.c_void_p(self.stream.cuda_stream),
                                                             C.byref(handle)))
        self.net = handle
        n = C.c_int64()
        _check_mlp(self.lib, self.net, self.lib.tufrg_mlp_nparams(self.net, C.byref(n)))
        self.nparams = n.value

    def params(self):
        t = self._torch
        out = t.empty(self.nparams, dtype=t.float32, device="cuda")
        _check_mlp(self.lib, self.net, self.lib.tufrg_mlp_get_params(self.net, C.c_void_p(out.data_ptr())))
        return out

    def set_params(self, p):
        _check_mlp(self.lib, self.net, self.lib.tufrg_mlp_set_params(
            self.net, _dev_array(p, self._torch.float32, self.nparams, "params")))

    def forward(self, x):
        t = self._torch
        rows = x.shape[0]
        _dev_array(x, t.float32, rows * self.widths[0], "x")
        y = t.empty((rows, self.widths[-1]), dtype=t.float32, device="cuda")
        _check_mlp(self.lib, self.net, self.lib.tufrg_mlp_forward(self.net, C.c_void_p(x.data_ptr()),
                                                                 C.c_void_p(y.data_ptr()), rows))
        return y

    def gradient(self, x, y):
        t = self._torch
        rows = x.shape[0]
        _dev_array(x, t.float32, rows * self.widths[0], "x")
        _dev_array(y, t.float32, rows * self.widths[-1], "y")
        g = t.empty(self.nparams, dtype=t.float32, device="cuda")
        loss = C.c_double()
        _check_mlp(self.lib, self.net, self.lib.tufrg_mlp_gradient(
            self.net, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), rows,
            C.c_void_p(g.data_ptr()), C.byref(loss)))
        return g, loss.value

    def train(self, x, y, steps: int, batch: int, lr: float, seed: int = 0):
        """Adam steps on minibatches of (x, y); returns the per-step losses."""
        import numpy as np
        t = self._torch
        rows = x.shape[0]
        _dev_array(x, t.float32, rows * self.widths[0], "x")
        _dev_array(y, t.float32, rows * self.widths[-1], "y")
        hist = (C.c_double * max(steps, 1))()
        _check_mlp(self.lib, self.net, self.lib.tufrg_mlp_train(
            self.net, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), rows, steps, batch,
            C.c_float(lr), C.c_uint64(seed), hist))
        return np.array(hist[:steps])

    def close(self):
        if getattr(self, "net", None):
            self.lib.tufrg_mlp_free(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mu_from_filling(t: float, tp: float, n: float, T: float, L: int = 1024) -> float:
    """Chemical potential for filling n (native host routine)."""
    lib = load_library()
    out = C.c_double()
    _check(lib, None, lib.tufrg_mu_from_filling(t, tp, n, T, L, C.byref(out)))
    return out.value


@dataclasses.dataclass
class FlowOptions:
    T0: float = 10.0
    Tmin: float = 0.01
    Xmax: float = 20.0
    scheme: str = "rk4"
    nsteps: int = 200
    rtol: float = 1e-7
    atol: float = 1e-9
    h0: float = 0.0
    max_steps: int = 0
    use_graph: bool = False


@dataclasses.dataclass
class FlowResult:
    status: str
    Tc: Optional[float]
    channel: Optional[str]
    q_index: Optional[int]
    irrep: Optional[str]
    max_abs_X: float
    n_rhs: int
    n_steps: int
    max_abs_V: float = float("nan")


class Context:
    """A set of model points with their device tables and workspace.

    points: objects with attributes t, tp, mu, U, Lq, Lk, shells.
    Arrays are torch float64 CUDA tensors laid out [channels][S]
    (channel-major, then point blocks [Nq][Nff][Nff]).
    regulator: "T" (temperature flow) or "omega" (Omega cutoff at zero
    temperature; every scale argument named T is then Omega).
    symmetric_state: the states passed in are C4v-symmetric (every state of
    a flow started at zero is); the inverse transform and the products then
    run at one transfer momentum per point-group orbit and the results are
    copied to the rest of the orbit by the form factors' signed permutations.
    """

    def __init__(self, points: Sequence, precision: str = "fp64", no_cross: bool = False,
                 stream=None, autotune: bool = False, loop_queue: bool = False,
                 no_symmetry: bool = False, fuse: bool = True, regulator: str = "T",
                 symmetric_state: bool = False, dense_projection: bool = False, loop_reuse: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise TufrgError("a GPU is required (torch.cuda.is_available() is False)")
        self._torch = torch
        self.lib = load_library()
        n = len(points)
        arr = (_Point * n)()
        for i, p in enumerate(points):
            if p.mu is None:
                raise TufrgError("point has no mu; solve mu_from_filling first")
            arr[i] = _Point(p.t, p.tp, p.mu, p.U, p.Lq, p.Lk, p.shells, 0)
        opt = _Options(PRECISIONS[precision],
                       (NO_CROSS if no_cross else 0) | (AUTOTUNE if autotune else 0)
                       | (LOOP_QUEUE if loop_queue else 0) | (NO_SYMMETRY if no_symmetry else 0)
                       | (0 if fuse else NO_FUSE) | REGULATORS[regulator]
                       | (SYMMETRIC_STATE if symmetric_state else 0)
                       | (DENSE_PROJECTION if dense_projection else 0)
                       | (0 if loop_reuse else NO_LOOP_REUSE))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        handle = C.c_void_p()
        meshes = [getattr(p, "mesh", None) for p in points]
        if any(m is not None for m in meshes):
            # non-uniform transfer meshes (host arrays, copied by the init call)
            import numpy as np
            keep = []
            marr = (_Mesh * n)()
            for i, m in enumerate(meshes):
                if m is None:
                    continue
                cols = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (m.qx, m.qy, m.w)]
                keep.append(cols)
                dpp = C.POINTER(C.c_double)
                marr[i] = _Mesh(len(cols[0]), *(c.ctypes.data_as(dpp) for c in cols))
            st = self.lib.tufrg_init_mesh(arr, marr, n, C.byref(opt), C.c_void_p(self.stream.cuda_stream),
                                          C.byref(handle))
        else:
            st = self.lib.tufrg_init(arr, n, C.byref(opt), C.c_void_p(self.stream.cuda_stream), C.byref(handle))
        _check(self.lib, None, st)
        self.ctx = handle
        self.npts = n
        self.layouts = []
        for i in range(n):
            off, nq, nff, tot = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64()
            _check(self.lib, self.ctx, self.lib.tufrg_layout(self.ctx, i, C.byref(off), C.byref(nq),
                                                             C.byref(nff), C.byref(tot)))
            self.layouts.append((off.value, nq.value, nff.value))
            self.S = tot.value

    def geometry(self, point: int = 0):
        """Loop kernel: (row slices per momentum, row chunks per column, block size, persistent)."""
        ns, nc, th, pe = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(self.lib, self.ctx, self.lib.tufrg_geometry(self.ctx, point, C.byref(ns), C.byref(nc),
                                                           C.byref(th), C.byref(pe)))
        return ns.value, nc.value, th.value, bool(pe.value)

    # ---------------------------------------------------------------- helpers
    def _T(self, T) -> "C.Array":
        Ts = [float(T)] * self.npts if not hasattr(T, "__len__") else [float(x) for x in T]
        return (C.c_double * self.npts)(*Ts)

    def _dev(self, x, nch: int):
        t = self._torch
        if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == t.float64 and x.is_contiguous()):
            raise TufrgError("expected a contiguous float64 CUDA tensor")
        if x.numel() != nch * self.S:
            raise TufrgError(f"expected {nch} x {self.S} elements, got {x.numel()}")
        return C.c_void_p(x.data_ptr())

    def empty(self, nch: int):
        return self._torch.empty((nch, self.S), dtype=self._torch.float64, device="cuda")

    def view(self, arr, point: int = 0):
        """[nch][S] array -> [nch][Nq][Nff][Nff] view of one point."""
        off, nq, nff = self.layouts[point]
        return arr.view(arr.shape[0], -1)[:, off:off + nq * nff * nff].reshape(arr.shape[0], nq, nff, nff)

    # ------------------------------------------------------------------ calls
    def bubbles(self, T, out=None):
        out = self.empty(2) if out is None else out
        _check(self.lib, self.ctx, self.lib.tufrg_bubbles(self.ctx, self._T(T), self._dev(out, 2)))
        return out

    def project(self, X, out=None):
        out = self.empty(3) if out is None else out
        _check(self.lib, self.ctx, self.lib.tufrg_project(self.ctx, self._dev(X, 3), self._dev(out, 3)))
        return out

    def rhs(self, T, X, out=None):
        out = self.empty(3) if out is None else out
        _check(self.lib, self.ctx, self.lib.tufrg_rhs(self.ctx, self._T(T), self._dev(X, 3),
                                                      self._dev(out, 3)))
        return out

    def rhs_noalloc(self, T, X, out):
        """tufrg_rhs_noalloc: the right-hand side with the library's static workspace."""
        _check(self.lib, self.ctx, self.lib.tufrg_rhs_noalloc(self.ctx, self._T(T), self._dev(X, 3),
                                                              self._dev(out, 3)))
        return out

    def sync(self):
        _check(self.lib, self.ctx, self.lib.tufrg_sync(self.ctx))

    def symmetry_defect(self, X) -> float:
        """Largest relative deviation of X from the C4v covariance law."""
        out = C.c_double()
        _check(self.lib, self.ctx, self.lib.tufrg_symmetry_defect(self.ctx, self._dev(X, 3), C.byref(out)))
        return out.value

    def flop_count(self):
        out = (C.c_double * 3)()
        _check(self.lib, self.ctx, self.lib.tufrg_flop_count(self.ctx, out))
        return {"loops": out[0], "projections": out[1], "products": out[2]}

    def loop_kernel_time(self, T, reps: int = 50):
        """(average microseconds of the loop kernel alone, its flops per launch)."""
        us, fl = C.c_double(), C.c_double()
        _check(self.lib, self.ctx, self.lib.tufrg_loop_kernel_time(self.ctx, self._T(T), reps, C.byref(us),
                                                                   C.byref(fl)))
        return us.value, fl.value

    KERNEL_STAGES = ("forward_transform", "bond_basis", "gather", "inverse_transform", "products")

    def kernel_times(self, T, X, out, reps: int = 50):
        """{stage: (average microseconds per launch, algorithmic flops per launch)} of the
        projection kernels and the products, each timed alone on one right-hand side's data
        (the products write dX/dT into out)."""
        us, fl = (C.c_double * 5)(), (C.c_double * 5)()
        _check(self.lib, self.ctx, self.lib.tufrg_kernel_times(self.ctx, self._T(T), self._dev(X, 3),
                                                               self._dev(out, 3), reps, us, fl))
        return {k: (us[i], fl[i]) for i, k in enumerate(self.KERNEL_STAGES)}

    def flow(self, X, opts: FlowOptions, raise_nonfinite: bool = False) -> List[FlowResult]:
        o = _FlowOpts(opts.T0, opts.Tmin, opts.Xmax, SCHEMES[opts.scheme], opts.nsteps, opts.rtol,
                      opts.atol, opts.h0, opts.max_steps, int(opts.use_graph))
        res = (_FlowResult * self.npts)()
        st = self.lib.tufrg_flow(self.ctx, C.byref(o), self._dev(X, 3), res)
        if st != -4 or raise_nonfinite:
            _check(self.lib, self.ctx, st)
        out = []
        for r in res:
            div = r.status == 1
            out.append(FlowResult(FLOW_STATUS.get(r.status, str(r.status)), r.Tc if div else None,
                                  CHANNELS[r.channel] if div else None, r.q_index if div else None,
                                  IRREPS[r.irrep] if div else None, r.max_abs_X, r.n_rhs, r.n_steps,
                                  max_abs_V=r.max_abs_V))
        return out

    # ------------------------------------------------------------- surrogate
    def harmonics(self, point: int = 0):
        """(N_S', table [N_S'][6] = (Sx, Sy, Ra_x, Ra_y, Rb_x, Rb_y), offset in harmonic arrays)."""
        import numpy as np
        n, off = C.c_int32(), C.c_int64()
        _check(self.lib, self.ctx, self.lib.tufrg_harmonics(self.ctx, point, C.byref(n), None, C.byref(off)))
        tab = (C.c_int32 * (6 * n.value))()
        _check(self.lib, self.ctx, self.lib.tufrg_harmonics(self.ctx, point, C.byref(n), tab, None))
        return n.value, np.array(tab[:], dtype=np.int32).reshape(n.value, 6), off.value

    def harmonics_length(self) -> int:
        total = 0
        for i in range(self.npts):
            n, _, _ = self.harmonics(i)
            total += self.layouts[i][1] * 2 * n
        return total

    def loop_harmonics(self, T):
        t = self._torch
        out = t.empty(self.harmonics_length(), dtype=t.float64, device="cuda")
        _check(self.lib, self.ctx, self.lib.tufrg_loop_harmonics(self.ctx, self._T(T),
                                                                 C.c_void_p(out.data_ptr())))
        return out

    def surrogate_dataset(self, T, n: int, seed: int = 0, x=None, y=None, with_index: bool = False):
        t = self._torch
        x = t.empty((n, 9), dtype=t.float32, device="cuda") if x is None else x
        y = t.empty((n, 4), dtype=t.float32, device="cuda") if y is None else y
        idx = t.empty((n, 3), dtype=t.int32, device="cuda") if with_index else None
        _check(self.lib, self.ctx, self.lib.tufrg_surrogate_dataset(
            self.ctx, self._T(T), n, C.c_uint64(seed), _dev_array(x, t.float32, 9 * n, "x"),
            _dev_array(y, t.float32, 4 * n, "y"), C.c_void_p(idx.data_ptr()) if with_index else None))
        return (x, y, idx) if with_index else (x, y)

    def attach_surrogate(self, a: "MLP", b: Optional["MLP"] = None, tol: float = 1e-3, check_stride: int = 8):
        """One network (b None) or an ensemble of two."""
        self._surrogates = (a, b)      # keep the networks alive while attached
        _check(self.lib, self.ctx, self.lib.tufrg_surrogate_attach(self.ctx, a.net, b.net if b is not None else None,
                                                                   tol, check_stride))

    def detach_surrogate(self):
        _check(self.lib, self.ctx, self.lib.tufrg_surrogate_attach(self.ctx, None, None, 0.0, 0))
        self._surrogates = None

    def surrogate_stats(self):
        out = (C.c_int64 * 3)()
        _check(self.lib, self.ctx, self.lib.tufrg_surrogate_stats(self.ctx, out))
        return {"exact_q": out[0], "queried_q": out[1], "failed_checks": out[2]}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.tufrg_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
