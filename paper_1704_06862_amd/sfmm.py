"""ctypes binding of libsfmm.so: argument marshalling only.

Every function here has the name of the C entry point it wraps (see
include/sfmm.h) and forwards plain pointers and sizes.  Vectors are complex128
numpy arrays (host, on_device=0) or torch complex128 CUDA tensors (device,
on_device=1, ordered on the context's stream).  There is no fallback: if the
HIP library is missing the import fails.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfmm.so")

SFMM_OK = 0
STATUS = {0: "SFMM_OK", 1: "SFMM_E_INVALID_ARG", 2: "SFMM_E_MESH", 3: "SFMM_E_OOM", 4: "SFMM_E_DEVICE",
          5: "SFMM_E_NOT_CONVERGED", 6: "SFMM_E_BREAKDOWN", 7: "SFMM_E_UNSUPPORTED"}
PREC_FP32, PREC_BF16_SPLIT, PREC_FP64 = 0, 1, 2
PART_NEAR, PART_FAR, PART_ALL = 1, 2, 3
PRECOND_ILU0, PRECOND_NONE, PRECOND_BLOCK_JACOBI, PRECOND_POLY = 0, 1, 2, 3
FORM_PMCHWT, FORM_JMCFIE, FORM_CNF = 0, 1, 2
SOLVER_GMRES, SOLVER_BICGSTAB, SOLVER_CGS = 0, 1, 2

EXPORTED = ["sfmm_default_options", "sfmm_setup", "sfmm_destroy", "sfmm_last_error", "sfmm_set_stream",
            "sfmm_num_unknowns", "sfmm_edges", "sfmm_matvec", "sfmm_precond", "sfmm_planewave_rhs",
            "sfmm_solve", "sfmm_rcs", "sfmm_near_rows", "sfmm_describe", "sfmm_product_bytes", "sfmm_profile",
            "sfmm_guess_default_options", "sfmm_guess_fit", "sfmm_guess_predict", "sfmm_mlp_train",
            "sfmm_solve_bodies", "sfmm_set_solver", "sfmm_span_predict", "sfmm_set_krylov", "sfmm_rcs_noalloc"]


class sfmm_body(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("vertices", ctypes.POINTER(ctypes.c_double)),
                ("n_triangles", ctypes.c_int32), ("triangles", ctypes.POINTER(ctypes.c_int32)),
                ("tri_regions", ctypes.POINTER(ctypes.c_int32)), ("n_regions", ctypes.c_int32),
                ("eps_r", ctypes.POINTER(ctypes.c_double)), ("mu_r", ctypes.POINTER(ctypes.c_double)),
                ("frequency_hz", ctypes.c_double)]


class sfmm_options(ctypes.Structure):
    _fields_ = [("finest_box", ctypes.c_double), ("n_levels", ctypes.c_int32), ("digits", ctypes.c_double),
                ("extra_multipoles", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("gmres_restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("device", ctypes.c_int32), ("verbose", ctypes.c_int32), ("preconditioner", ctypes.c_int32),
                ("poly_degree", ctypes.c_int32), ("graphs", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("kernel_plan", ctypes.c_int32), ("formulation", ctypes.c_int32), ("quad_points", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("ilu_pivot_tol", ctypes.c_double),
                ("setup_on_device", ctypes.c_int32)]


class sfmm_solve_info(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("guess_used", ctypes.c_int32), ("true_residual", ctypes.c_double),
                ("initial_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class sfmm_guess_options(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("harmonics", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("lr", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32)]


class SfmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def load():
    try:
        # torch ships its own ROCm runtime; loading it first makes the library
        # bind to the same libamdhip64 instead of a second copy
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_1704_06862_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.sfmm_default_options.argtypes = [ctypes.POINTER(sfmm_options)]
    lib.sfmm_default_options.restype = None
    lib.sfmm_setup.argtypes = [ctypes.POINTER(sfmm_body), I32, ctypes.POINTER(sfmm_options), ctypes.POINTER(P)]
    lib.sfmm_destroy.argtypes = [P]
    lib.sfmm_destroy.restype = None
    lib.sfmm_last_error.argtypes = [P]
    lib.sfmm_last_error.restype = ctypes.c_char_p
    lib.sfmm_set_stream.argtypes = [P, P]
    lib.sfmm_num_unknowns.argtypes = [P, I32, ctypes.POINTER(I64)]
    lib.sfmm_edges.argtypes = [P, I32, P]
    lib.sfmm_matvec.argtypes = [P, I32, I32, P, P, I32, I32]
    lib.sfmm_precond.argtypes = [P, I32, I32, P, P, I32]
    lib.sfmm_planewave_rhs.argtypes = [P, I32, I32, P, P, P, I32]
    lib.sfmm_solve.argtypes = [P, I32, I32, P, P, P, P, I32]
    lib.sfmm_rcs.argtypes = [P, I32, I32, P, I32, P, P, I32]
    lib.sfmm_near_rows.argtypes = [P, I32, I32, P, P]
    lib.sfmm_describe.argtypes = [P, I32, P, P]
    lib.sfmm_profile.argtypes = [P, I32, P, P]
    lib.sfmm_product_bytes.argtypes = [P, I32, P]
    lib.sfmm_guess_default_options.argtypes = [ctypes.POINTER(sfmm_guess_options)]
    lib.sfmm_guess_default_options.restype = None
    lib.sfmm_guess_fit.argtypes = [P, I32, I32, P, P, P, ctypes.POINTER(sfmm_guess_options), P, I32]
    lib.sfmm_guess_predict.argtypes = [P, I32, I32, P, P, P, I32]
    lib.sfmm_mlp_train.argtypes = [I32, I32, P, P, I32, P, P, I32, D, P, P, P]
    lib.sfmm_solve_bodies.argtypes = [P, I32, P, P, P, P, P, I32]
    lib.sfmm_set_solver.argtypes = [P, I32, I32, D]
    lib.sfmm_set_krylov.argtypes = [P, I32]
    lib.sfmm_span_predict.argtypes = [P, I32, I32, P, P, P, I32]
    lib.sfmm_rcs_noalloc.argtypes = [P, I32, I32, P, I32, P, P]
    for name in EXPORTED:
        if name not in ("sfmm_default_options", "sfmm_destroy", "sfmm_last_error", "sfmm_guess_default_options"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _check(status, ctx=None):
    if status != SFMM_OK:
        msg = lib().sfmm_last_error(ctx)
        raise SfmmError(status, msg.decode() if msg else "")


def _ptr(a):
    """Data pointer of a numpy array or torch tensor, and whether it is on the GPU."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data, 0
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), 1 if a.is_cuda else 0
    raise TypeError(type(a))


def _override(o, overrides):
    names = {f[0] for f in type(o)._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r} for {type(o).__name__}")
        setattr(o, k, v)
    return o


def sfmm_default_options(**overrides):
    o = sfmm_options()
    lib().sfmm_default_options(ctypes.byref(o))
    return _override(o, overrides)


def sfmm_guess_default_options(**overrides):
    o = sfmm_guess_options()
    lib().sfmm_guess_default_options(ctypes.byref(o))
    return _override(o, overrides)


def sfmm_mlp_train(sizes, params, X, Y, steps=0, lr=1e-3, device=0):
    """Network kernels on their own.  params: float32 host array (updated in
    place when steps > 0).  Returns (loss history [steps + 1], gradient at the
    initial parameters, output at the initial parameters)."""
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    if params.dtype != np.float32 or not params.flags["C_CONTIGUOUS"]:
        raise ValueError("params must be a contiguous float32 array (updated in place)")
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    loss = np.zeros(steps + 1)
    grads = np.zeros_like(params)
    out = np.zeros((X.shape[0], int(sizes[-1])), dtype=np.float32)
    _check(lib().sfmm_mlp_train(device, len(sizes), sizes.ctypes.data, params.ctypes.data, X.shape[0],
                                X.ctypes.data, Y.ctypes.data, steps, lr, loss.ctypes.data, grads.ctypes.data,
                                out.ctypes.data))
    return loss, grads, out


class Context:
    """Owns an sfmm_ctx for a list of workloads.Body objects."""

    def __init__(self, bodies, **options):
        self._keep = []
        arr = (sfmm_body * len(bodies))()
        for i, b in enumerate(bodies):
            v = np.ascontiguousarray(b.vertices, dtype=np.float64)
            t = np.ascontiguousarray(b.triangles, dtype=np.int32)
            r = np.ascontiguousarray(b.tri_regions, dtype=np.int32)
            eps = np.ascontiguousarray(np.stack([np.real(b.eps_r), np.imag(b.eps_r)], 1), dtype=np.float64)
            mu = np.ascontiguousarray(np.stack([np.real(b.mu_r), np.imag(b.mu_r)], 1), dtype=np.float64)
            self._keep += [v, t, r, eps, mu]
            arr[i] = sfmm_body(len(v), v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(t),
                               t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(b.eps_r),
                               eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(b.frequency))
        self.options = sfmm_default_options(**options)
        ctx = ctypes.c_void_p()
        _check(lib().sfmm_setup(arr, len(bodies), ctypes.byref(self.options), ctypes.byref(ctx)), None)
        self.ctx = ctx
        self._keep = []
        self.n_bodies = len(bodies)

    def close(self):
        if getattr(self, "ctx", None):
            lib().sfmm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- thin wrappers ------------------------------------------------------
    def sfmm_set_stream(self, stream_ptr):
        _check(lib().sfmm_set_stream(self.ctx, ctypes.c_void_p(stream_ptr)), self.ctx)

    def sfmm_num_unknowns(self, body=0):
        n = ctypes.c_int64()
        _check(lib().sfmm_num_unknowns(self.ctx, body, ctypes.byref(n)), self.ctx)
        return n.value

    def sfmm_edges(self, body=0):
        ne = self.sfmm_num_unknowns(body) // 2
        out = np.zeros((ne, 2), dtype=np.int32)
        _check(lib().sfmm_edges(self.ctx, body, out.ctypes.data), self.ctx)
        return out

    def _vec(self, a, n_rhs, body, name):
        """Pointer and location of a block of n_rhs complex128 vectors of the
        body's 2E unknowns; the library reads or writes exactly that many
        numbers, so the size is checked here."""
        if isinstance(a, np.ndarray):
            ok = a.dtype == np.complex128
            size = a.size
        elif hasattr(a, "numel"):
            ok = str(a.dtype) == "torch.complex128"
            size = a.numel()
        else:
            raise TypeError(f"{name}: numpy array or torch tensor expected")
        if not ok:
            raise TypeError(f"{name} must be complex128")
        n = self.sfmm_num_unknowns(body)
        if size != n_rhs * n:
            raise ValueError(f"{name} must hold {n_rhs} x {n} complex numbers, not {size}")
        return _ptr(a)

    @staticmethod
    def _rows(a):
        if a.ndim not in (1, 2):
            raise ValueError("vectors are [n] or [n_rhs][n]")
        return a.shape[0] if a.ndim == 2 else 1

    def _vec_args(self, x, y, body):
        n_rhs = self._rows(x)
        px, dx = self._vec(x, n_rhs, body, "x")
        py, dy = self._vec(y, n_rhs, body, "y")
        if dx != dy:
            raise ValueError("x and y must both be host or both be device arrays")
        return px, py, dx, n_rhs

    def sfmm_matvec(self, x, y, body=0, parts=PART_ALL):
        px, py, dev, n_rhs = self._vec_args(x, y, body)
        _check(lib().sfmm_matvec(self.ctx, body, n_rhs, px, py, dev, parts), self.ctx)
        return y

    def sfmm_precond(self, x, y, body=0):
        px, py, dev, n_rhs = self._vec_args(x, y, body)
        _check(lib().sfmm_precond(self.ctx, body, n_rhs, px, py, dev), self.ctx)
        return y

    def sfmm_planewave_rhs(self, angles, b, pol=None, body=0):
        angles = np.ascontiguousarray(angles, dtype=np.float64).reshape(-1, 2)
        polv = None if pol is None else np.ascontiguousarray(pol, dtype=np.float64)
        pb, dev = self._vec(b, len(angles), body, "b")
        _check(lib().sfmm_planewave_rhs(self.ctx, body, len(angles), angles.ctypes.data,
                                        None if polv is None else polv.ctypes.data, pb, dev), self.ctx)
        return b

    def sfmm_solve(self, b, x, x0=None, body=0, raise_on_nonconvergence=False):
        pb, px, dev, n_rhs = self._vec_args(b, x, body)
        info = (sfmm_solve_info * n_rhs)()
        p0 = None
        if x0 is not None:
            p0, d0 = self._vec(x0, n_rhs, body, "x0")
            if d0 != dev:
                raise ValueError("x0 must be where b and x are")
        st = lib().sfmm_solve(self.ctx, body, n_rhs, pb, px, p0, info, dev)
        if st != SFMM_OK and (st != 5 or raise_on_nonconvergence):
            _check(st, self.ctx)
        return [dict(converged=bool(i.converged), iterations=i.iterations, restarts=i.restarts,
                     guess_used=bool(i.guess_used), true_residual=i.true_residual,
                     initial_residual=i.initial_residual, seconds=i.seconds) for i in info]

    def sfmm_set_solver(self, gmres_restart=0, max_iters=0, tol=0.0):
        _check(lib().sfmm_set_solver(self.ctx, gmres_restart, max_iters, tol), self.ctx)

    def sfmm_set_krylov(self, solver):
        _check(lib().sfmm_set_krylov(self.ctx, solver), self.ctx)

    def sfmm_solve_bodies(self, problems, raise_on_nonconvergence=False):
        """problems: list of (body, b, x); all host or all device arrays.
        Returns one list of info dicts per problem."""
        n = len(problems)
        bodies = np.array([p[0] for p in problems], dtype=np.int32)
        n_rhs = np.array([self._rows(p[1]) for p in problems], dtype=np.int32)
        devs = set()
        pb, px = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
        for i, (bi, b, x) in enumerate(problems):
            pb[i], d1 = self._vec(b, int(n_rhs[i]), bi, "b")
            px[i], d2 = self._vec(x, int(n_rhs[i]), bi, "x")
            devs.update((d1, d2))
        if len(devs) != 1:
            raise ValueError("all vectors must be host arrays or all device arrays")
        info = (sfmm_solve_info * int(n_rhs.sum()))()
        st = lib().sfmm_solve_bodies(self.ctx, n, bodies.ctypes.data, n_rhs.ctypes.data, pb, px, info, devs.pop())
        if st != SFMM_OK and (st != 5 or raise_on_nonconvergence):
            _check(st, self.ctx)
        out, k = [], 0
        for r in n_rhs:
            out.append([dict(converged=bool(i.converged), iterations=i.iterations, restarts=i.restarts,
                             guess_used=bool(i.guess_used), true_residual=i.true_residual,
                             initial_residual=i.initial_residual, seconds=i.seconds) for i in info[k:k + r]])
            k += r
        return out

    def sfmm_guess_fit(self, angles, x, pol=None, body=0, **options):
        """Train the learned initial guess on solutions x [n][2E] of the
        incidences angles [n][2]; returns the final training loss."""
        angles = np.ascontiguousarray(angles, dtype=np.float64).reshape(-1, 2)
        polv = None if pol is None else np.ascontiguousarray(pol, dtype=np.float64)
        px, dev = self._vec(x, len(angles), body, "x")
        go = sfmm_guess_default_options(**options)
        loss = ctypes.c_double(0.0)
        _check(lib().sfmm_guess_fit(self.ctx, body, len(angles), angles.ctypes.data,
                                    None if polv is None else polv.ctypes.data, px, ctypes.byref(go),
                                    ctypes.byref(loss), dev), self.ctx)
        return loss.value

    def sfmm_span_predict(self, angles, x0, pol=None, body=0):
        angles = np.ascontiguousarray(angles, dtype=np.float64).reshape(-1, 2)
        polv = None if pol is None else np.ascontiguousarray(pol, dtype=np.float64)
        px, dev = self._vec(x0, len(angles), body, "x0")
        _check(lib().sfmm_span_predict(self.ctx, body, len(angles), angles.ctypes.data,
                                       None if polv is None else polv.ctypes.data, px, dev), self.ctx)
        return x0

    def sfmm_guess_predict(self, angles, x0, pol=None, body=0):
        angles = np.ascontiguousarray(angles, dtype=np.float64).reshape(-1, 2)
        polv = None if pol is None else np.ascontiguousarray(pol, dtype=np.float64)
        px, dev = self._vec(x0, len(angles), body, "x0")
        _check(lib().sfmm_guess_predict(self.ctx, body, len(angles), angles.ctypes.data,
                                        None if polv is None else polv.ctypes.data, px, dev), self.ctx)
        return x0

    def sfmm_rcs(self, x, theta_phi, body=0):
        n_rhs = self._rows(x)
        px, dev = self._vec(x, n_rhs, body, "x")
        tp = np.ascontiguousarray(theta_phi, dtype=np.float64).reshape(-1, 2)
        sigma = np.zeros((n_rhs, len(tp), 2))
        _check(lib().sfmm_rcs(self.ctx, body, n_rhs, px, len(tp), tp.ctypes.data, sigma.ctypes.data, dev), self.ctx)
        return sigma

    def sfmm_rcs_noalloc(self, x, theta_phi, body=0):
        """x: device tensor [n_rhs][2E] complex128 (the call allocates no device memory)."""
        n_rhs = self._rows(x)
        px, dev = self._vec(x, n_rhs, body, "x")
        if not dev:
            raise ValueError("sfmm_rcs_noalloc takes device vectors")
        tp = np.ascontiguousarray(theta_phi, dtype=np.float64).reshape(-1, 2)
        sigma = np.zeros((n_rhs, len(tp), 2))
        _check(lib().sfmm_rcs_noalloc(self.ctx, body, n_rhs, px, len(tp), tp.ctypes.data, sigma.ctypes.data),
               self.ctx)
        return sigma

    def sfmm_near_rows(self, edges, body=0):
        edges = np.ascontiguousarray(edges, dtype=np.int32)
        n = self.sfmm_num_unknowns(body)
        out = np.zeros((len(edges), 2, n), dtype=np.complex128)
        _check(lib().sfmm_near_rows(self.ctx, body, len(edges), edges.ctypes.data, out.ctypes.data), self.ctx)
        return out

    def sfmm_describe(self, body=0):
        info = np.zeros(4, dtype=np.int64)
        trunc = np.zeros((8, 16), dtype=np.int32)
        _check(lib().sfmm_describe(self.ctx, body, info.ctypes.data, trunc.ctypes.data), self.ctx)
        return dict(levels=int(info[0]), finest_boxes=int(info[1]), near_pairs=int(info[2]),
                    translation_pairs=int(info[3]), truncation=trunc)

    def sfmm_product_bytes(self, body=0):
        b = np.zeros(8, dtype=np.int64)
        _check(lib().sfmm_product_bytes(self.ctx, body, b.ctypes.data), self.ctx)
        keys = ["near", "x_y", "patterns", "levels", "translation", "interpolation", "total"]
        return {k: int(v) for k, v in zip(keys, b)}

    def sfmm_profile(self, enable):
        t = np.zeros(8)
        n = np.zeros(8, dtype=np.int64)
        _check(lib().sfmm_profile(self.ctx, int(enable), t.ctypes.data, n.ctypes.data), self.ctx)
        return t, n
