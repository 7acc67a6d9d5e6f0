"""ctypes binding of libgplmm.so (the C ABI declared in include/gplmm.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Device vectors are torch CUDA tensors (float64, length N, cell-record
layout); the library works on torch's current stream.  There is no CPU
fallback: when the library is missing or no GPU is present the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgplmm.so")

GPLMM_FP64, GPLMM_FP32 = 0, 1
WIND = {"zero": 0, "stokes": 1, "caller": 2}
ERRORS = {-1: "bad argument", -2: "geometry", -3: "HIP error", -4: "breakdown", -5: "call order"}


class Options(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("h", ctypes.c_double), ("periodic", ctypes.c_int * 3),
                ("precision", ctypes.c_int), ("wind_mode", ctypes.c_int),
                ("tag_layers", ctypes.c_int), ("dual_dilations", ctypes.c_int),
                ("restart", ctypes.c_int), ("newton_tol", ctypes.c_double),
                ("lin_tol", ctypes.c_double), ("newton_maxit", ctypes.c_int),
                ("lin_maxit", ctypes.c_int), ("tile", ctypes.c_int), ("host_only", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("line_search", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("build_matrix", ctypes.c_int), ("split_tiles", ctypes.c_int),
                ("mg_form", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("red_blocks", ctypes.c_int), ("stencil_block", ctypes.c_int), ("trsv_mode", ctypes.c_int),
                ("from_cache", ctypes.c_int), ("t_reduction_ms", ctypes.c_double),
                ("t_stencil_ms", ctypes.c_double), ("t_trsv_ms", ctypes.c_double)]


class Layout(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("nrec", ctypes.c_int), ("ncell", ctypes.c_int64),
                ("N", ctypes.c_int64), ("nface_active", ctypes.c_int64), ("Np", ctypes.c_int),
                ("Nc", ctypes.c_int), ("Ny", ctypes.c_int), ("pin", ctypes.c_int64),
                ("ndual_cells", ctypes.c_int64), ("local_unknowns", ctypes.c_int64),
                ("factor_bytes", ctypes.c_int64), ("ncolors", ctypes.c_int), ("lu_flops", ctypes.c_double),
                ("nsplit", ctypes.c_int), ("sep_unknowns", ctypes.c_int64), ("nfblock", ctypes.c_int),
                ("max_fblock", ctypes.c_int), ("f_unknowns", ctypes.c_int64)]


class CoarseOptions(ctypes.Structure):
    _fields_ = [("increments", ctypes.c_int), ("newton_maxit", ctypes.c_int), ("tol", ctypes.c_double)]


class CoarseStats(ctypes.Structure):
    _fields_ = [("increments", ctypes.c_int), ("newton_its", ctypes.c_int * 64), ("rc_rel", ctypes.c_double * 64),
                ("fine_rel_residual", ctypes.c_double), ("t_build_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("converged", ctypes.c_int)]

    def as_dict(self):
        n = self.increments
        return dict(increments=n, newton_its=[self.newton_its[k] for k in range(n)],
                    rc_rel=[self.rc_rel[k] for k in range(n)], fine_rel_residual=self.fine_rel_residual,
                    t_build_ms=self.t_build_ms, t_total_ms=self.t_total_ms, converged=bool(self.converged))


class Stats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int), ("lin_its_total", ctypes.c_int),
                ("lin_its", ctypes.c_int * 64), ("res_hist", ctypes.c_double * 65),
                ("r0_norm", ctypes.c_double), ("t_build_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("builds", ctypes.c_int), ("converged", ctypes.c_int), ("gs_reorth", ctypes.c_int),
                ("step_length", ctypes.c_double * 64), ("t_coarse_ms", ctypes.c_double),
                ("learned_builds", ctypes.c_int), ("coarse_fallbacks", ctypes.c_int)]

    def as_dict(self):
        n = self.newton_its
        return dict(newton_its=n, lin_its_total=self.lin_its_total,
                    lin_its=[self.lin_its[k] for k in range(n)],
                    res_hist=[self.res_hist[k] for k in range(n + 1)],
                    r0_norm=self.r0_norm, t_build_ms=self.t_build_ms, t_solve_ms=self.t_solve_ms,
                    t_total_ms=self.t_total_ms, builds=self.builds, converged=bool(self.converged),
                    gs_reorth=self.gs_reorth, step_length=[self.step_length[k] for k in range(n)],
                    t_coarse_ms=self.t_coarse_ms, learned_builds=self.learned_builds,
                    coarse_fallbacks=self.coarse_fallbacks)


EXPORTS = ["gplmm_default_options", "gplmm_setup", "gplmm_setup_batch", "gplmm_batch_info",
           "gplmm_sample_residuals", "gplmm_layout_info", "gplmm_get_maps",
           "gplmm_get_duals", "gplmm_get_subdomains", "gplmm_get_split", "gplmm_get_fblocks", "gplmm_continuation", "gplmm_residual", "gplmm_matvec", "gplmm_build_matvec", "gplmm_build",
           "gplmm_precond_apply", "gplmm_get_coarse", "gplmm_newton_solve", "gplmm_set_timing", "gplmm_kernel_time",
           "gplmm_reset_timers", "gplmm_last_error", "gplmm_destroy",
           "gplmm_mlp_create", "gplmm_mlp_num_params", "gplmm_mlp_set_params", "gplmm_mlp_get_params",
           "gplmm_mlp_forward", "gplmm_mlp_grad", "gplmm_mlp_adam", "gplmm_mlp_train", "gplmm_mlp_last_error",
           "gplmm_mlp_destroy", "gplmm_set_coarse_model", "gplmm_coarse_entries",
           "gplmm_autotune", "gplmm_set_tuning", "gplmm_set_progress", "gplmm_sample_residuals_noalloc",
           "gplmm_coarse_default_options", "gplmm_coarse_solve", "gplmm_setup_pnm"]

_lib = None

PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double)


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgplmm.so is not built; run __graft_entry__.build() or "
                           "python paper_2510_22077_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, None
    lib.gplmm_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.gplmm_default_options.restype = V
    lib.gplmm_setup.argtypes = [P, P, D, D, ctypes.POINTER(ctypes.c_double), D, ctypes.POINTER(Options),
                                ctypes.POINTER(ctypes.c_void_p)]
    lib.gplmm_setup.restype = I
    lib.gplmm_setup_pnm.argtypes = [P, P, P, D, D, ctypes.POINTER(ctypes.c_double), D, ctypes.POINTER(Options),
                                    ctypes.POINTER(ctypes.c_void_p)]
    lib.gplmm_setup_pnm.restype = I
    lib.gplmm_setup_batch.argtypes = [I, P, P, P, P, P, P, P, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p)]
    lib.gplmm_setup_batch.restype = I
    lib.gplmm_batch_info.argtypes = [P, ctypes.POINTER(ctypes.c_int), P, P, P, P]
    lib.gplmm_batch_info.restype = I
    lib.gplmm_sample_residuals.argtypes = [P, P, P, P]
    lib.gplmm_sample_residuals.restype = I
    lib.gplmm_sample_residuals_noalloc.argtypes = [P, P, P, P]
    lib.gplmm_sample_residuals_noalloc.restype = I
    lib.gplmm_coarse_default_options.argtypes = [ctypes.POINTER(CoarseOptions)]
    lib.gplmm_coarse_default_options.restype = V
    lib.gplmm_coarse_solve.argtypes = [P, ctypes.POINTER(CoarseOptions), P, ctypes.POINTER(CoarseStats)]
    lib.gplmm_coarse_solve.restype = I
    lib.gplmm_layout_info.argtypes = [P, ctypes.POINTER(Layout)]
    lib.gplmm_layout_info.restype = I
    lib.gplmm_get_maps.argtypes = [P, P, P, P, P, P]
    lib.gplmm_get_maps.restype = I
    lib.gplmm_get_duals.argtypes = [P, P, P]
    lib.gplmm_get_duals.restype = I
    lib.gplmm_get_subdomains.argtypes = [P, P, P]
    lib.gplmm_get_subdomains.restype = I
    lib.gplmm_get_split.argtypes = [P, I, P, P]
    lib.gplmm_get_split.restype = I
    lib.gplmm_get_fblocks.argtypes = [P, P, P]
    lib.gplmm_get_fblocks.restype = I
    lib.gplmm_continuation.argtypes = [P, I, P, P, P]
    lib.gplmm_continuation.restype = I
    for f in ("gplmm_residual", "gplmm_matvec"):
        getattr(lib, f).argtypes = [P, P, P, P]
        getattr(lib, f).restype = I
    lib.gplmm_build_matvec.argtypes = [P, P, P]
    lib.gplmm_build_matvec.restype = I
    lib.gplmm_build.argtypes = [P, P]
    lib.gplmm_build.restype = I
    lib.gplmm_get_coarse.argtypes = [P, P, P]
    lib.gplmm_get_coarse.restype = I
    lib.gplmm_precond_apply.argtypes = [P, P, P]
    lib.gplmm_precond_apply.restype = I
    lib.gplmm_newton_solve.argtypes = [P, P, P, ctypes.POINTER(Stats)]
    lib.gplmm_newton_solve.restype = I
    lib.gplmm_set_progress.argtypes = [P, PROGRESS_FN, P]
    lib.gplmm_set_progress.restype = I
    lib.gplmm_set_timing.argtypes = [P, I]
    lib.gplmm_set_timing.restype = I
    lib.gplmm_kernel_time.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
    lib.gplmm_kernel_time.restype = I
    lib.gplmm_reset_timers.argtypes = [P]
    lib.gplmm_reset_timers.restype = V
    lib.gplmm_last_error.argtypes = [P]
    lib.gplmm_last_error.restype = ctypes.c_char_p
    lib.gplmm_destroy.argtypes = [P]
    lib.gplmm_destroy.restype = V
    D = ctypes.c_double
    lib.gplmm_mlp_create.argtypes = [I, I, I, I, I, P, ctypes.POINTER(P)]
    lib.gplmm_mlp_create.restype = I
    lib.gplmm_mlp_num_params.argtypes = [P]
    lib.gplmm_mlp_num_params.restype = ctypes.c_int64
    for f in ("gplmm_mlp_set_params", "gplmm_mlp_get_params"):
        getattr(lib, f).argtypes = [P, P]
        getattr(lib, f).restype = I
    lib.gplmm_mlp_forward.argtypes = [P, P, I, P]
    lib.gplmm_mlp_forward.restype = I
    lib.gplmm_mlp_grad.argtypes = [P, P, P, I, ctypes.POINTER(D), P]
    lib.gplmm_mlp_grad.restype = I
    lib.gplmm_mlp_adam.argtypes = [P, D, D, D, D]
    lib.gplmm_mlp_adam.restype = I
    lib.gplmm_mlp_train.argtypes = [P, P, P, I, I, I, D, ctypes.POINTER(D)]
    lib.gplmm_mlp_train.restype = I
    lib.gplmm_mlp_last_error.argtypes = [P]
    lib.gplmm_mlp_last_error.restype = ctypes.c_char_p
    lib.gplmm_mlp_destroy.argtypes = [P]
    lib.gplmm_mlp_destroy.restype = V
    lib.gplmm_set_coarse_model.argtypes = [P, P]
    lib.gplmm_set_coarse_model.restype = I
    lib.gplmm_coarse_entries.argtypes = [P, ctypes.POINTER(ctypes.c_int64), P, P, P, P, P]
    lib.gplmm_coarse_entries.restype = I
    lib.gplmm_autotune.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(Tuning)]
    lib.gplmm_autotune.restype = I
    lib.gplmm_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.gplmm_set_tuning.restype = I
    _lib = lib
    return lib


class GplmmError(RuntimeError):
    pass


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Solver:
    """One gplmm context (one sample, one stream)."""

    def __init__(self, mask, labels, rho=1.0, mu=1.0, body=(1.0, 0.0, 0.0), dt=0.0, groups=None, **kw):
        """groups: pore labels for the pore-network decomposition (gplmm_setup_pnm), in which
        ``labels`` are the throat regions; None for the pore decomposition (gplmm_setup)."""
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        labels = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
        if mask.ndim == 2:
            mask = mask[None]
            labels = labels[None]
        if mask.shape != labels.shape:
            raise ValueError("mask and labels must have the same shape")
        nz, ny, nx = mask.shape
        o = self._prepare(nx, ny, nz, **kw)
        b = (ctypes.c_double * 3)(*[float(v) for v in body])
        ctx = ctypes.c_void_p()
        if groups is None:
            rc = self.lib.gplmm_setup(mask.ctypes.data, labels.ctypes.data, float(rho), float(mu), b, float(dt),
                                      ctypes.byref(o), ctypes.byref(ctx))
        else:
            grp = np.ascontiguousarray(np.asarray(groups, dtype=np.int32).reshape(mask.shape))
            self._groups = grp
            rc = self.lib.gplmm_setup_pnm(mask.ctypes.data, labels.ctypes.data, grp.ctypes.data, float(rho),
                                          float(mu), b, float(dt), ctypes.byref(o), ctypes.byref(ctx))
        self._finish(ctx, rc, "gplmm_setup")
        self.shape = mask.shape

    def _prepare(self, nx, ny, nz, h=1.0, periodic=(1, 0, 0), precision="fp64", wind="stokes", tag_layers=1,
                 dual_dilations=-1, restart=30, newton_tol=1e-8, lin_tol=1e-9, newton_maxit=30, lin_maxit=600,
                 host_only=False, stream=None, line_search=False, use_graph=True, build_matrix="geometric",
                 split_tiles=0, mg_form=0):
        lib = load()
        self.lib = lib
        self.ctx = ctypes.c_void_p()
        o = Options()
        lib.gplmm_default_options(ctypes.byref(o))
        o.nx, o.ny, o.nz = nx, ny, nz
        o.h = h
        for k in range(3):
            o.periodic[k] = int(periodic[k])
        o.precision = GPLMM_FP32 if precision == "fp32" else GPLMM_FP64
        o.wind_mode = WIND[wind]
        o.tag_layers = tag_layers
        o.dual_dilations = dual_dilations
        o.restart = restart
        o.newton_tol = newton_tol
        o.lin_tol = lin_tol
        o.newton_maxit = newton_maxit
        o.lin_maxit = lin_maxit
        o.host_only = 1 if host_only else 0
        o.line_search = 1 if line_search else 0
        o.use_graph = 1 if use_graph else 0
        o.build_matrix = {"geometric": 0, "jacobian": 1}[build_matrix]
        o.split_tiles = int(split_tiles)
        o.mg_form = int(mg_form)
        self.torch = None
        if not host_only:
            import torch
            if not torch.cuda.is_available():
                raise GplmmError("no GPU: the gPLMM library runs on the device only")
            self.torch = torch
            if stream is None:
                stream = torch.cuda.current_stream()
            o.stream = ctypes.c_void_p(stream.cuda_stream)
            self.stream = stream
        return o

    def _finish(self, ctx, rc, what):
        lib = self.lib
        self.ctx = ctx
        if rc != 0:
            msg = lib.gplmm_last_error(ctx).decode() if ctx.value else ""
            if ctx.value:
                lib.gplmm_destroy(ctx)
                self.ctx = ctypes.c_void_p()
            raise GplmmError("%s failed (%d, %s): %s" % (what, rc, ERRORS.get(rc, "?"), msg))
        L = Layout()
        lib.gplmm_layout_info(ctx, ctypes.byref(L))
        self.layout = L
        self.N = L.N

    def batch_info(self):
        """Per-sample offsets: cells, voxels, primaries, interfaces (nsamples + 1 each)."""
        ns = ctypes.c_int()
        self._check(self.lib.gplmm_batch_info(self.ctx, ctypes.byref(ns), None, None, None, None), "batch_info")
        n = ns.value
        out = dict(cell_off=np.zeros(n + 1, np.int64), voxel_off=np.zeros(n + 1, np.int64),
                   prim_off=np.zeros(n + 1, np.int32), iface_off=np.zeros(n + 1, np.int32))
        self._check(self.lib.gplmm_batch_info(self.ctx, ctypes.byref(ns), *[a.ctypes.data for a in out.values()]),
                    "batch_info")
        out["nsamples"] = n
        return out

    def sample_residuals(self, x, x_prev=None):
        """||r_s(x)|| / ||r_s(0)|| of every sample (host array)."""
        n = self.batch_info()["nsamples"]
        out = np.zeros(n)
        self._check(self.lib.gplmm_sample_residuals(self.ctx, _ptr(self._vec(x)), _ptr(self._vec(x_prev)),
                                                    out.ctypes.data), "sample_residuals")
        return out

    def sample_residuals_noalloc(self, x, out, x_prev=None):
        """The same norms written to the caller's device FP64 tensor ``out`` (one entry per
        sample) by the allocation-free entry point; no synchronisation."""
        n = self.batch_info()["nsamples"]
        if out.dtype != self.torch.float64 or not out.is_cuda or out.numel() < n or not out.is_contiguous():
            raise ValueError("out must be a contiguous device float64 tensor of >= %d entries" % n)
        self._check(self.lib.gplmm_sample_residuals_noalloc(self.ctx, _ptr(self._vec(x)), _ptr(self._vec(x_prev)),
                                                            _ptr(out)), "sample_residuals_noalloc")
        return out

    # ---- housekeeping
    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.gplmm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc < 0:
            raise GplmmError("%s failed (%d, %s): %s" % (what, rc, ERRORS.get(rc, "?"),
                                                         self.lib.gplmm_last_error(self.ctx).decode()))
        return rc

    def info(self):
        L = self.layout
        return {f: getattr(L, f) for f, _ in Layout._fields_}

    def maps(self):
        L = self.layout
        out = dict(cell_voxel=np.zeros(L.ncell, np.int32), cell_iface=np.zeros(L.ncell, np.int32),
                   cell_prim=np.zeros(L.ncell, np.int32), face_owner=np.zeros(L.N, np.int32),
                   face_tag=np.zeros(L.N, np.int8))
        self._check(self.lib.gplmm_get_maps(self.ctx, *[a.ctypes.data for a in out.values()]), "get_maps")
        return out

    def duals(self):
        ptr = np.zeros(self.layout.Nc + 1, np.int64)
        self.lib.gplmm_get_duals(self.ctx, ptr.ctypes.data, None)
        cells = np.zeros(max(int(ptr[-1]), 1), np.int32)
        self.lib.gplmm_get_duals(self.ctx, ptr.ctypes.data, cells.ctypes.data)
        return [cells[ptr[j]:ptr[j + 1]].copy() for j in range(self.layout.Nc)]

    def subdomains(self):
        """(n, factor_elems) of every local problem: primaries, then dual grids."""
        k = self.layout.Np + self.layout.Nc
        n = np.zeros(max(k, 1), np.int32)
        fe = np.zeros(max(k, 1), np.int64)
        self._check(self.lib.gplmm_get_subdomains(self.ctx, n.ctypes.data, fe.ctypes.data), "get_subdomains")
        return n[:k], fe[:k]

    def splits(self):
        """Nested-dissection plans: a list of dicts (prim, nA, nB, nS, slots in the order
        [A, B, S])."""
        out = []
        for k in range(self.layout.nsplit):
            info = np.zeros(4, np.int32)
            self._check(self.lib.gplmm_get_split(self.ctx, k, info.ctypes.data, None), "get_split")
            slots = np.zeros(int(info[1] + info[2] + info[3]), np.int32)
            self._check(self.lib.gplmm_get_split(self.ctx, k, info.ctypes.data, slots.ctypes.data), "get_split")
            out.append(dict(prim=int(info[0]), nA=int(info[1]), nB=int(info[2]), nS=int(info[3]), slots=slots))
        return out

    def fblocks(self):
        """Blocks of A^f_f for the back-substitution of Eq. xf (mg_form 1, 2): a list of
        arrays of record slots, one per block."""
        ptr = np.zeros(self.layout.nfblock + 1, np.int64)
        slots = np.zeros(max(int(self.layout.f_unknowns), 1), np.int32)
        self._check(self.lib.gplmm_get_fblocks(self.ctx, ptr.ctypes.data, slots.ctypes.data), "get_fblocks")
        return [slots[ptr[k]:ptr[k + 1]].copy() for k in range(self.layout.nfblock)]

    # ---- device vectors
    def zeros(self):
        return self.torch.zeros(self.N, dtype=self.torch.float64, device="cuda")

    def _vec(self, t):
        if t is None:
            return None
        if not (t.is_cuda and t.dtype == self.torch.float64 and t.is_contiguous() and t.numel() == self.N):
            raise ValueError("expected a contiguous float64 CUDA tensor of length %d" % self.N)
        return t

    def residual(self, x, x_prev=None, out=None):
        out = self.zeros() if out is None else out
        self._check(self.lib.gplmm_residual(self.ctx, _ptr(self._vec(x)), _ptr(self._vec(x_prev)),
                                            _ptr(self._vec(out))), "residual")
        return out

    def matvec(self, xlin, v, out=None):
        out = self.zeros() if out is None else out
        self._check(self.lib.gplmm_matvec(self.ctx, _ptr(self._vec(xlin)), _ptr(self._vec(v)),
                                          _ptr(self._vec(out))), "matvec")
        return out

    def build_matvec(self, v, out=None):
        out = self.zeros() if out is None else out
        self._check(self.lib.gplmm_build_matvec(self.ctx, _ptr(self._vec(v)), _ptr(self._vec(out))),
                    "build_matvec")
        return out

    def build(self, wind=None):
        self._check(self.lib.gplmm_build(self.ctx, _ptr(self._vec(wind))), "build")

    def coarse_operator(self):
        """Host copy of the assembled coarse operator Rhat X Phat (after build)."""
        n = ctypes.c_int()
        self.lib.gplmm_get_coarse(self.ctx, None, ctypes.byref(n))
        A = np.zeros((n.value, n.value))
        self._check(self.lib.gplmm_get_coarse(self.ctx, A.ctypes.data, None), "get_coarse")
        return A

    def coarse_entries(self, exact=True):
        """Pattern, features, scales (and exact values of the last exact build) of the
        coarse operator's entries."""
        n = ctypes.c_int64()
        self._check(self.lib.gplmm_coarse_entries(self.ctx, ctypes.byref(n), None, None, None, None, None),
                    "coarse_entries")
        k = n.value
        rows, cols = np.zeros(k, np.int32), np.zeros(k, np.int32)
        feat, scale = np.zeros((k, 16), np.float32), np.zeros(k, np.float32)
        ex = np.zeros(k) if exact else None
        self._check(self.lib.gplmm_coarse_entries(self.ctx, ctypes.byref(n), rows.ctypes.data, cols.ctypes.data,
                                                  feat.ctypes.data, scale.ctypes.data,
                                                  ex.ctypes.data if exact else None), "coarse_entries")
        return dict(rows=rows, cols=cols, feat=feat, scale=scale, exact=ex)

    def autotune(self, cache_path=None):
        """Pick the launch parameters of the hot kernels by measurement (see gplmm_autotune)."""
        t = Tuning()
        self._check(self.lib.gplmm_autotune(self.ctx, cache_path.encode() if cache_path else None,
                                            ctypes.byref(t)), "autotune")
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def set_tuning(self, red_blocks=1024, stencil_block=256, trsv_mode=0):
        t = Tuning(red_blocks, stencil_block, trsv_mode, 0, 0.0, 0.0, 0.0)
        self._check(self.lib.gplmm_set_tuning(self.ctx, ctypes.byref(t)), "set_tuning")

    def set_coarse_model(self, mlp):
        self._check(self.lib.gplmm_set_coarse_model(self.ctx, mlp.m if mlp is not None else None),
                    "set_coarse_model")
        self._coarse_model = mlp   # keep it alive while the context uses it

    def precond_apply(self, v, out=None):
        out = self.zeros() if out is None else out
        self._check(self.lib.gplmm_precond_apply(self.ctx, _ptr(self._vec(v)), _ptr(self._vec(out))),
                    "precond_apply")
        return out

    def newton_solve(self, x0=None, x_prev=None):
        x = self.zeros() if x0 is None else self._vec(x0).clone()
        st = Stats()
        rc = self._check(self.lib.gplmm_newton_solve(self.ctx, _ptr(self._vec(x_prev)), _ptr(x),
                                                     ctypes.byref(st)), "newton_solve")
        d = st.as_dict()
        d["rc"] = rc
        return x, d

    def continuation(self, scales, x0=None):
        """Reynolds-number continuation (gplmm_continuation): the body force raised through
        the given fractions (increasing, ending at 1); returns (x, [stats of each step], rc)."""
        sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64))
        x = self.zeros() if x0 is None else self._vec(x0).clone()
        sts = (Stats * len(sc))()
        rc = self.lib.gplmm_continuation(self.ctx, len(sc), sc.ctypes.data, _ptr(x), sts)
        if rc < 0:
            self._check(rc, "continuation")
        return x, [sts[k].as_dict() for k in range(len(sc))], rc

    def coarse_solve(self, increments=1, newton_maxit=50, tol=1e-6):
        """Coarse-scale solver (gplmm_coarse_solve): returns (x, stats)."""
        o = CoarseOptions()
        self.lib.gplmm_coarse_default_options(ctypes.byref(o))
        o.increments, o.newton_maxit, o.tol = int(increments), int(newton_maxit), float(tol)
        x = self.zeros()
        st = CoarseStats()
        rc = self.lib.gplmm_coarse_solve(self.ctx, ctypes.byref(o), _ptr(x), ctypes.byref(st))
        if rc < 0:
            self._check(rc, "coarse_solve")
        return x, st.as_dict()

    def set_progress(self, fn=None):
        """fn(newton_it, lin_its, rel) after every FGMRES cycle (rel = -1) and Newton step."""
        if fn is None:
            self._progress = None
            return self._check(self.lib.gplmm_set_progress(self.ctx, PROGRESS_FN(), None), "set_progress")
        self._progress = PROGRESS_FN(lambda user, k, its, rel: fn(k, its, rel))
        return self._check(self.lib.gplmm_set_progress(self.ctx, self._progress, None), "set_progress")

    def set_timing(self, on=True):
        self.lib.gplmm_set_timing(self.ctx, 1 if on else 0)

    def kernel_time(self, name):
        ms, by = ctypes.c_double(), ctypes.c_double()
        n = self.lib.gplmm_kernel_time(self.ctx, name.encode(), ctypes.byref(ms), ctypes.byref(by))
        return dict(samples=n, avg_ms=ms.value, bytes=by.value)

    def reset_timers(self):
        self.lib.gplmm_reset_timers(self.ctx)



class BatchSolver(Solver):
    """Many independent samples in one gplmm context: one block-diagonal system whose
    subdomains are all factorised and solved in the same launches."""

    def __init__(self, masks, labels, rho=1.0, mu=1.0, bodies=None, dt=None, **kw):
        ns = len(masks)
        if ns < 1 or len(labels) != ns:
            raise ValueError("need one label image per mask")
        ms, ls, dims = [], [], []
        for m, l in zip(masks, labels):
            m = np.ascontiguousarray(np.asarray(m, dtype=np.uint8))
            l = np.ascontiguousarray(np.asarray(l, dtype=np.int32))
            if m.ndim == 2:
                m, l = m[None], l[None]
            if m.shape != l.shape:
                raise ValueError("mask and labels must have the same shape")
            ms.append(m)
            ls.append(l)
            dims += [m.shape[2], m.shape[1], m.shape[0]]
        o = self._prepare(dims[0], dims[1], dims[2], **kw)
        per = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (ns,)))
        rho_a, mu_a = per(rho), per(mu)
        dt_a = per(0.0 if dt is None else dt)
        if bodies is None:
            bodies = [(1.0, 0.0, 0.0)] * ns
        body_a = np.zeros((ns, 3))
        for s_, b in enumerate(bodies):
            body_a[s_, :len(b)] = b
        mptr = (ctypes.c_void_p * ns)(*[m.ctypes.data for m in ms])
        lptr = (ctypes.c_void_p * ns)(*[l.ctypes.data for l in ls])
        dims_a = np.asarray(dims, dtype=np.int32)
        self._keep = (ms, ls, rho_a, mu_a, dt_a, body_a, dims_a)
        ctx = ctypes.c_void_p()
        rc = self.lib.gplmm_setup_batch(ns, mptr, lptr, dims_a.ctypes.data, rho_a.ctypes.data, mu_a.ctypes.data,
                                        body_a.ctypes.data, dt_a.ctypes.data, ctypes.byref(o), ctypes.byref(ctx))
        self._finish(ctx, rc, "gplmm_setup_batch")
        self.shapes = [m.shape for m in ms]

    def split(self, x):
        """Per-sample slices of a batch vector (views)."""
        off = self.batch_info()["cell_off"] * self.layout.nrec
        return [x[off[k]:off[k + 1]] for k in range(len(off) - 1)]


class Mlp:
    """The BF16 matrix-core MLP of the library (learned coarse coefficients).

    Parameters are exchanged as a flat FP32 array in the packed layout of
    ``gplmm_mlp_num_params``: per layer W (fan_in x fan_out, row-major), then b."""

    def __init__(self, nin, nhidden=128, nlayers=3, nout=1, max_batch=4096):
        import torch
        self.torch = torch
        self.lib = load()
        self.nin, self.nout = nin, nout
        self.m = ctypes.c_void_p()
        rc = self.lib.gplmm_mlp_create(nin, nhidden, nlayers, nout, max_batch, None, ctypes.byref(self.m))
        if rc != 0:
            raise GplmmError("gplmm_mlp_create failed (%d)" % rc)

    def _check(self, rc, what):
        if rc < 0:
            raise GplmmError("%s: %s (%d)" % (what, self.lib.gplmm_mlp_last_error(self.m).decode(), rc))
        return rc

    def _f32(self, t):
        t = self.torch.as_tensor(t, dtype=self.torch.float32, device="cuda")
        return t.contiguous()

    def num_params(self):
        return int(self.lib.gplmm_mlp_num_params(self.m))

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.num_params()
        self._check(self.lib.gplmm_mlp_set_params(self.m, a.ctypes.data), "mlp_set_params")

    def get_params(self):
        a = np.zeros(self.num_params(), np.float32)
        self._check(self.lib.gplmm_mlp_get_params(self.m, a.ctypes.data), "mlp_get_params")
        return a

    def forward(self, x):
        x = self._f32(x)
        y = self.torch.empty((x.shape[0], self.nout), dtype=self.torch.float32, device="cuda")
        self._check(self.lib.gplmm_mlp_forward(self.m, _ptr(x), x.shape[0], _ptr(y)), "mlp_forward")
        return y

    def grad(self, x, t):
        x, t = self._f32(x), self._f32(t)
        loss = ctypes.c_double()
        g = np.zeros(self.num_params(), np.float32)
        self._check(self.lib.gplmm_mlp_grad(self.m, _ptr(x), _ptr(t), x.shape[0], ctypes.byref(loss),
                                            g.ctypes.data), "mlp_grad")
        return loss.value, g

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self._check(self.lib.gplmm_mlp_adam(self.m, lr, b1, b2, eps), "mlp_adam")

    def train(self, x, t, epochs=10, batch=1024, lr=1e-3):
        x, t = self._f32(x), self._f32(t)
        loss = ctypes.c_double()
        self._check(self.lib.gplmm_mlp_train(self.m, _ptr(x), _ptr(t), x.shape[0], epochs, batch, lr,
                                             ctypes.byref(loss)), "mlp_train")
        return loss.value

    def close(self):
        if self.m:
            self.lib.gplmm_mlp_destroy(self.m)
            self.m = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
