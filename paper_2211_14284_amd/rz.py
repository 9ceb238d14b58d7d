"""ctypes binding of ``librz.so`` (include/rz.h).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  Device vectors are
passed as torch tensors (their data pointers) on the context's stream.

There is no fallback: if the shared library is missing, importing this module
raises.
"""
import atexit
import ctypes
import sys
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librz.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2211_14284_amd.build`")
lib = ctypes.CDLL(LIB_PATH)

GRAD, CURL, DIV = 0, 1, 2
SPACES = {"grad": GRAD, "curl": CURL, "div": DIV}
F64, F32, BF16 = 0, 1, 2
COEF_CONST, COEF_CELL, COEF_SAMPLES = 0, 1, 2
PREC_F64, PREC_MIXED, PREC_DEFECT = 0, 1, 2
EXPORT_DOFMAP, EXPORT_PATCH, EXPORT_IC_PATTERN, EXPORT_IC_FACTOR = 0, 1, 2, 3
EXPORT_TABLES1D, EXPORT_AUXCOEF, EXPORT_OMEGA, EXPORT_PATCH_KERNEL = 4, 5, 6, 7
EXPORT_EDGE_PATCH, EXPORT_STATS, EXPORT_PAPER_DIAG, EXPORT_AUTOTUNE, EXPORT_GRAPHS, EXPORT_HMG = 8, 9, 10, 11, 12, 13
AUX_CELL_AVG, AUX_PAPER_DIAG = 0, 1
PATCH_IC, PATCH_CHOLESKY = 0, 1
NORM_2, NORM_NATURAL = 0, 1
DECOMP_SC, DECOMP_FULL, DECOMP_SC_VERTEX, DECOMP_FULL_PH = 0, 1, 2, 3
COARSE_DIRECT, COARSE_HMG = 0, 1
KERNELS = ("apply", "condense", "patch", "expand", "transfer", "coarse", "krylov")
STATUS = {0: "RZ_OK", -1: "RZ_ERR_ARG", -2: "RZ_ERR_OOM", -3: "RZ_ERR_BREAKDOWN",
          -4: "RZ_ERR_NOT_CONVERGED", -5: "RZ_ERR_HIP", -6: "RZ_ERR_SINGULAR", -7: "RZ_ERR_NODEVICE"}


class RzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("vertex_xyz", ctypes.POINTER(ctypes.c_double)), ("dirichlet_faces", ctypes.c_uint32)]


class Coef(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("alpha", ctypes.POINTER(ctypes.c_double)),
                ("beta", ctypes.POINTER(ctypes.c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("space", ctypes.c_int32), ("p", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("rtol", ctypes.c_double), ("omega", ctypes.c_double),
                ("lanczos_seed", ctypes.c_uint64), ("hdiv_eps", ctypes.c_double), ("aux", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("patch_solver", ctypes.c_int32),
                ("decomposition", ctypes.c_int32), ("norm", ctypes.c_int32), ("coarse", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("omega", ctypes.c_double), ("t_solve_ms", ctypes.c_double), ("iters_natural", ctypes.c_int32)]


_vp = ctypes.c_void_p
_proto = {
    "rz_opts_default": (None, [ctypes.POINTER(Opts)]),
    "rz_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "rz_destroy": (ctypes.c_int, [_vp]),
    "rz_last_error": (ctypes.c_char_p, [_vp]),
    "rz_setup": (ctypes.c_int, [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Coef), ctypes.POINTER(Opts),
                                ctypes.POINTER(_vp)]),
    "rz_free": (ctypes.c_int, [_vp]),
    "rz_sizes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "rz_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int32]),
    "rz_apply_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    "rz_relax": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int32]),
    "rz_prolong_add": (ctypes.c_int, [_vp, _vp, _vp]),
    "rz_restrict": (ctypes.c_int, [_vp, _vp, _vp]),
    "rz_coarse_solve": (ctypes.c_int, [_vp, _vp, _vp]),
    "rz_vcycle": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32]),
    "rz_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(SolveInfo)]),
    "rz_export": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int64, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "rz_sync": (ctypes.c_int, [_vp]),
    "rz_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "rz_set_graph": (ctypes.c_int, [_vp, ctypes.c_int]),
    "rz_timing_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "rz_aux_data": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "rz_solve_batched": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(_vp),
                                        ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(SolveInfo)]),
    "rz_set_aux": (ctypes.c_int, [_vp, _vp]),
    "rz_hodge_create": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, ctypes.c_int32, ctypes.POINTER(_vp)]),
    "rz_hodge_free": (ctypes.c_int, [_vp]),
    "rz_hodge_sizes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "rz_hodge_apply": (ctypes.c_int, [_vp, _vp, _vp]),
    "rz_hodge_precond": (ctypes.c_int, [_vp, _vp, _vp]),
    "rz_hodge_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(SolveInfo)]),
    "rz_mlp_create": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.POINTER(_vp)]),
    "rz_mlp_free": (ctypes.c_int, [_vp]),
    "rz_mlp_last_error": (ctypes.c_char_p, [_vp]),
    "rz_mlp_nparams": (ctypes.c_int64, [_vp]),
    "rz_mlp_params": (ctypes.c_int, [_vp, _vp, ctypes.c_int32]),
    "rz_mlp_predict": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64]),
    "rz_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), _vp]),
    "rz_mlp_adam_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_float]),
    "rz_mlp_train": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                    ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
}
for _name, (_res, _args) in _proto.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


# Every object that holds a library handle.  At interpreter exit (before module
# teardown) the problems and MLPs are freed, then the contexts, so no device
# buffer, pinned buffer or event outlives the Python objects into the HIP
# runtime's own teardown.
_live = weakref.WeakSet()


def close_all():
    """Free every live Hodge solver, then every problem and MLP, then every context
    (also run at exit)."""
    objs = list(_live)
    for rank in (0, 1, 2):
        for o in objs:
            if (2 if isinstance(o, Context) else 0 if isinstance(o, Hodge) else 1) == rank:
                try:
                    o.close()
                except RzError:
                    pass


atexit.register(close_all)


def _nrhs(t, nrhs=None):
    """Right-hand sides of a multi-vector: the second extent of an (ndofs, nrhs)
    tensor (DoF-major, right-hand side fastest), 1 for a vector; an explicit
    nrhs for int addresses."""
    if nrhs is not None:
        return int(nrhs)
    if t is None or isinstance(t, int) or t.dim() == 1:
        return 1
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError("multi-vectors are contiguous (ndofs, nrhs) tensors")
    return int(t.shape[1])


def _ptr(t):
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


class Context:
    """A library context on one HIP device (device=-1: host-only, symbolic setup)."""

    def __init__(self, device=0, stream=None):
        self.handle = _vp()
        sp = None
        if device >= 0 and stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        code = lib.rz_create(ctypes.byref(self.handle), device, sp)
        if code != 0:
            raise RzError(code, "rz_create failed")
        self.device = device
        # the stream must outlive the context (and the problems, which hold the context)
        self._stream = stream
        _live.add(self)

    def error(self):
        return lib.rz_last_error(self.handle).decode()

    def check(self, code):
        if code != 0:
            raise RzError(code, self.error())

    def close(self):
        """Destroy the context (its problems and MLPs must be closed first)."""
        if self.handle:
            self.check(lib.rz_destroy(self.handle))
            self.handle = _vp()

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check usable when module globals are gone
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def default_opts(**kw):
    o = Opts()
    lib.rz_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "space" and isinstance(v, str):
            v = SPACES[v]
        setattr(o, k, v)
    return o


class Problem:
    """One discretised Riesz map: ``Problem(ctx, n, p, alpha, beta, ...)``.

    n: cells per axis (int or 3-tuple); alpha, beta: scalars (constant), arrays of
    one value per cell, or (ncells, 27) arrays of reference samples; vertices:
    optional (n_vertices, 3) array (any trilinear mesh).  Further keywords set the
    fields of rz_opts (precision, maxit, rtol, omega, hdiv_eps, aux, graph, ...).
    """

    def __init__(self, ctx, n, p, alpha=1.0, beta=1.0, space="grad", vertices=None,
                 dirichlet=0x3F, **opts):
        self.ctx = ctx
        nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
        self._keep = []
        vp = None
        if vertices is not None:
            v = np.ascontiguousarray(vertices, dtype=np.float64).ravel()
            self._keep.append(v)
            vp = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        mesh = Mesh(nx, ny, nz, vp, dirichlet)
        a = np.ascontiguousarray(np.atleast_1d(alpha), dtype=np.float64)
        b = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
        nc = nx * ny * nz
        if a.ndim == 2 or b.ndim == 2:
            # 27 samples per cell (reference points {-1,0,1}^3, x fastest)
            kind = COEF_SAMPLES
            a = np.ascontiguousarray(np.broadcast_to(a.reshape(-1, 27) if a.ndim == 2 else a[:, None],
                                                     (nc, 27))).ravel()
            b = np.ascontiguousarray(np.broadcast_to(b.reshape(-1, 27) if b.ndim == 2 else b[:, None],
                                                     (nc, 27))).ravel()
        else:
            kind = COEF_CONST if (a.size == 1 and b.size == 1) else COEF_CELL
            if kind == COEF_CELL:
                a = np.ascontiguousarray(np.broadcast_to(a, (nc,)))
                b = np.ascontiguousarray(np.broadcast_to(b, (nc,)))
        self._keep += [a, b]
        coef = Coef(kind, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        o = default_opts(space=space, p=p, **opts)
        self.handle = _vp()
        ctx.check(lib.rz_setup(ctx.handle, ctypes.byref(mesh), ctypes.byref(coef), ctypes.byref(o),
                               ctypes.byref(self.handle)))
        s = (ctypes.c_int64 * 8)()
        ctx.check(lib.rz_sizes(self.handle, s))
        (self.ndofs, self.nfree, self.ncells, self.nslots, self.ncoarse, self.nnz, self.nrows,
         self.npatches) = list(s)
        self.n = (nx, ny, nz)
        self.p = p
        _live.add(self)

    # ---- compute (device tensors) -------------------------------------------------
    def apply(self, x, y, dtype=F64, nrhs=None):
        """y = A x; x, y: (ndofs,) or (ndofs, nrhs) device tensors."""
        self.ctx.check(lib.rz_apply(self.handle, _ptr(x), _ptr(y), dtype, _nrhs(x, nrhs)))

    def apply_noalloc(self, x, y, dtype=F64):
        """y = A x with the library's static workspace (no allocation in the call)."""
        self.ctx.check(lib.rz_apply_noalloc(self.handle, _ptr(x), _ptr(y), dtype))

    def relax(self, r, z, dtype=F64, nrhs=None):
        """z = M^{-1} r; r, z: (ndofs,) or (ndofs, nrhs) device tensors."""
        self.ctx.check(lib.rz_relax(self.handle, _ptr(r), _ptr(z), dtype, _nrhs(r, nrhs)))

    def prolong_add(self, xc, xf):
        self.ctx.check(lib.rz_prolong_add(self.handle, _ptr(xc), _ptr(xf)))

    def restrict(self, rf, rc):
        self.ctx.check(lib.rz_restrict(self.handle, _ptr(rf), _ptr(rc)))

    def coarse_solve(self, rc, xc):
        self.ctx.check(lib.rz_coarse_solve(self.handle, _ptr(rc), _ptr(xc)))

    def vcycle(self, r, z, nrhs=None):
        self.ctx.check(lib.rz_vcycle(self.handle, _ptr(r), _ptr(z), _nrhs(r, nrhs)))

    def sync(self):
        """Wait for the queued work; raises if a coarse-solve wait gave up."""
        self.ctx.check(lib.rz_sync(self.handle))

    def solve(self, b, x, check=True, nrhs=None):
        """Solve A x = b.  b, x: (ndofs,) device tensors (returns a SolveInfo) or
        (ndofs, nrhs) multi-vectors (returns a list of nrhs SolveInfo)."""
        k = _nrhs(b, nrhs)
        infos = (SolveInfo * k)()
        code = lib.rz_solve(self.handle, _ptr(b), _ptr(x), k, infos)
        if check:
            self.ctx.check(code)
        if k == 1 and (nrhs is None and (b is None or isinstance(b, int) or b.dim() == 1)):
            return infos[0]
        return [infos[r] for r in range(k)]

    def set_graph(self, on=True):
        """Run CG iterations from captured HIP graphs (rz_opts.graph) or not."""
        self.ctx.check(lib.rz_set_graph(self.handle, 1 if on else 0))

    # ---- per-kernel device timing --------------------------------------------------
    def timing(self, on=True):
        self.ctx.check(lib.rz_timing_enable(self.handle, 1 if on else 0))

    def timing_read(self):
        """{kernel: (total ms, launches)} accumulated since the last read."""
        ms = (ctypes.c_double * len(KERNELS))()
        cnt = (ctypes.c_int64 * len(KERNELS))()
        self.ctx.check(lib.rz_timing_read(self.handle, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}

    # ---- exports (host numpy arrays) ----------------------------------------------
    def _export(self, what, index=0, dtype=np.float64):
        nb = ctypes.c_int64(0)
        self.ctx.check(lib.rz_export(self.handle, what, index, None, ctypes.byref(nb)))
        buf = np.empty(nb.value // np.dtype(dtype).itemsize, dtype=dtype)
        self.ctx.check(lib.rz_export(self.handle, what, index, buf.ctypes.data_as(_vp), ctypes.byref(nb)))
        return buf

    def dofmap(self):
        m = self._export(EXPORT_DOFMAP, dtype=np.int64)
        return m.reshape(self.ncells, -1)

    def patch(self, k):
        v = self._export(EXPORT_PATCH, k, dtype=np.int64)
        return int(v[0]), v[1:]

    def edge_patch(self, k):
        """(edge id, DoFs) of non-empty edge-star patch k (H(curl); H(div): its
        NCE_p potential problem)."""
        v = self._export(EXPORT_EDGE_PATCH, k, dtype=np.int64)
        return int(v[0]), v[1:]

    def stats(self):
        """{factor_nnz, patch_rows}: lower non-zeros and rows of the IC factors of all
        non-empty vertex patches (H(grad))."""
        v = self._export(EXPORT_STATS, dtype=np.int64)
        return {"factor_nnz": int(v[0]), "patch_rows": int(v[1])}

    def ic_pattern(self, k):
        return self._export(EXPORT_IC_PATTERN, k, dtype=np.int32).reshape(-1, 2)

    def ic_factor(self, k):
        return self._export(EXPORT_IC_FACTOR, k)

    def tables1d(self):
        p = self.p
        v = self._export(EXPORT_TABLES1D)
        n1 = p + 1
        o = 0
        out = {}
        for name, size, shape in (("lam", p - 1, (p - 1,)), ("B", n1 * n1, (n1, n1)), ("A", n1 * n1, (n1, n1)),
                                  ("D", p * n1, (p, n1)), ("E", n1 * 2, (n1, 2))):
            out[name] = v[o:o + size].reshape(shape)
            o += size
        return out

    def paper_diagonals(self, cell):
        """(dm, da): the broken diagonals of one cell (RZ_AUX_PAPER_DIAG problems)."""
        v = self._export(EXPORT_PAPER_DIAG, cell)
        n1 = self.p + 1
        return v[:n1 ** 3], v[n1 ** 3:].reshape(3, -1)

    def autotune(self):
        """{"f64"|"f32": {"candidates": [(cap, ms), ...], "chosen": cap}} of the
        streaming patch solve's setup autotuner (empty where the register kernel runs)."""
        v = self._export(EXPORT_AUTOTUNE)
        out, o = {}, 0
        for name in ("f64", "f32"):
            n = int(v[o])
            cand = [(int(v[o + 1 + 2 * k]), float(v[o + 2 + 2 * k])) for k in range(n)]
            out[name] = {"candidates": cand, "chosen": int(v[o + 1 + 2 * n])}
            o += 2 + 2 * n
        return out

    def graph_stats(self):
        """(captures, iterations replayed, segments per captured iteration) of the
        captured CG iterations (graph=1)."""
        return tuple(int(v) for v in self._export(EXPORT_GRAPHS, dtype=np.int64))

    def hmg_levels(self):
        """Free vertices per level of the h-multigrid coarse solver (coarse=COARSE_HMG),
        finest first."""
        return [int(v) for v in self._export(EXPORT_HMG, dtype=np.int64)]

    def aux_coefficients(self):
        return self._export(EXPORT_AUXCOEF).reshape(self.ncells, 6)

    def aux_data(self):
        """(targets, features, base): the least-squares fit of the separable weights
        to the broken diagonals, the 51 per-cell features and the weights in use."""
        t = np.zeros((self.ncells, 6))
        f = np.zeros((self.ncells, 51))
        b = np.zeros((self.ncells, 6))
        self.ctx.check(lib.rz_aux_data(self.handle, t.ctypes.data, f.ctypes.data, b.ctypes.data))
        return t, f, b

    def set_aux(self, coef6):
        c = np.ascontiguousarray(coef6, dtype=np.float64).reshape(self.ncells, 6)
        self.ctx.check(lib.rz_set_aux(self.handle, c.ctypes.data))

    def omega(self):
        return float(self._export(EXPORT_OMEGA)[0])

    def patch_kernel(self):
        """(FP64, FP32): 1 where the patch solve holds the factor in registers."""
        v = self._export(EXPORT_PATCH_KERNEL, dtype=np.int32)
        return int(v[0]), int(v[1])

    def close(self):
        if self.handle:
            lib.rz_free(self.handle)
            self.handle = _vp()

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check usable when module globals are gone
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Hodge:
    """Mixed Hodge Laplacian k in {1, 2, 3} on two set-up problems (rz_hodge_*):
    ``Hodge(k, lo, hi, cheb_steps=4)`` with lo of form degree k-1 and hi of degree k
    (None for k = 3), both with dirichlet=0.  Vectors are [sigma; u] of length
    n_lo + n_hi."""

    def __init__(self, k, lo, hi=None, cheb_steps=4):
        self.ctx, self.lo, self.hi = lo.ctx, lo, hi
        self.handle = _vp()
        self.ctx.check(lib.rz_hodge_create(k, lo.handle, hi.handle if hi is not None else None, cheb_steps,
                                           ctypes.byref(self.handle)))
        s = (ctypes.c_int64 * 2)()
        e = (ctypes.c_double * 4)()
        self.ctx.check(lib.rz_hodge_sizes(self.handle, s, e))
        self.n_lo, self.n_hi = int(s[0]), int(s[1])
        self.eig = list(e)
        _live.add(self)

    def apply(self, x, y):
        self.ctx.check(lib.rz_hodge_apply(self.handle, _ptr(x), _ptr(y)))

    def precond(self, r, z):
        self.ctx.check(lib.rz_hodge_precond(self.handle, _ptr(r), _ptr(z)))

    def solve(self, b, x, rtol=1e-8, maxit=500, check=True):
        info = SolveInfo()
        code = lib.rz_hodge_solve(self.handle, _ptr(b), _ptr(x), rtol, maxit, ctypes.byref(info))
        if check:
            self.ctx.check(code)
        return info

    def close(self):
        if self.handle:
            lib.rz_hodge_free(self.handle)
            self.handle = _vp()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def solve_batched(problems, bs, xs, check=True):
    """Batched solves: problems[i] solves the device tensor bs[i] ((ndofs,) or
    (ndofs, nrhs): the same nrhs for every problem) into xs[i]; problems on
    different contexts run concurrently.  Returns an (n, nrhs) list of SolveInfo."""
    n = len(problems)
    nrhs = _nrhs(bs[0]) if n else 1
    H = (_vp * n)(*[p.handle for p in problems])
    B = (_vp * n)(*[_ptr(b) for b in bs])
    X = (_vp * n)(*[_ptr(x) for x in xs])
    infos = (SolveInfo * max(1, n * nrhs))()
    code = lib.rz_solve_batched(H, n, B, X, nrhs, infos)
    if check and code != 0:
        raise RzError(code, "rz_solve_batched failed")
    return [[infos[i * nrhs + r] for r in range(nrhs)] for i in range(n)]


class MLP:
    """The library's small MLP (FP32 on the context's device): nin -> nhid (tanh) ->
    nhid (tanh) -> nout.  Arrays passed to predict/train are torch tensors on the
    device; parameters move as packed host float32 arrays."""

    def __init__(self, ctx, nin=51, nhid=64, nout=6, seed=1234):
        self.ctx = ctx
        self.handle = _vp()
        self._check(lib.rz_mlp_create(ctx.handle, nin, nhid, nout, seed, ctypes.byref(self.handle)))
        self.nin, self.nhid, self.nout = nin, nhid, nout
        self.nparams = int(lib.rz_mlp_nparams(self.handle))
        _live.add(self)

    def _check(self, code):
        if code != 0:
            msg = lib.rz_mlp_last_error(self.handle).decode() if getattr(self, "handle", None) else ""
            raise RzError(code, msg)

    def params(self):
        p = np.zeros(self.nparams, dtype=np.float32)
        self._check(lib.rz_mlp_params(self.handle, p.ctypes.data, 0))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        self._check(lib.rz_mlp_params(self.handle, p.ctypes.data, 1))

    def predict(self, X, Y):
        self._check(lib.rz_mlp_predict(self.handle, _ptr(X), _ptr(Y), X.shape[0]))

    def loss_grad(self, X, Y):
        loss = ctypes.c_double()
        g = np.zeros(self.nparams, dtype=np.float32)
        self._check(lib.rz_mlp_loss_grad(self.handle, _ptr(X), _ptr(Y), X.shape[0], ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def adam_step(self, X, Y, lr):
        self._check(lib.rz_mlp_adam_step(self.handle, _ptr(X), _ptr(Y), X.shape[0], lr))

    def train(self, X, Y, epochs, batch, lr, seed=7):
        loss = ctypes.c_double()
        self._check(lib.rz_mlp_train(self.handle, _ptr(X), _ptr(Y), X.shape[0], epochs, batch, lr, seed,
                                     ctypes.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "handle", None):
            lib.rz_mlp_free(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check usable when module globals are gone
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
