"""ctypes binding of libpngf (argument marshalling only).

Every computation runs inside libpngf: its host precompute and its HIP
kernels.  PyTorch only provides the device workspace (one uint8 tensor) and
the HIP stream.  The module fails loudly when libpngf.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpngf.so")

PNGF_FP64_PLAIN = 0
PNGF_MIXED = 1
PNGF_RFORM = 2
PNGF_FLAG_TIMING = 1
PNGF_FLAG_STEP_LAUNCHES = 2
PNGF_FLAG_TIMING_STEPS = 4
PNGF_FLAG_PIVOT_SEARCH = 8
PNGF_PIXEL_DIELECTRIC = 0
PNGF_PIXEL_PEC = 1

KERNEL_IDS = {"score": 0, "select": 1, "accept": 2, "lu": 3, "other": 4, "fold": 5,
              "mixed_q": 6, "wood": 7, "tile": 8}

_STATUS = {0: "OK", -1: "EINVAL", -2: "ESINGULAR", -3: "ENUMERIC", -4: "EDEVICE",
           -5: "ESTATE", -6: "ENOMEM"}


class PngfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pngf {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("npml", C.c_int32),
                ("h", C.c_double),
                ("eps_static", C.POINTER(C.c_double)),
                ("design_mask", C.POINTER(C.c_uint8)),
                ("eps_lo", C.c_double), ("eps_hi", C.c_double),
                ("nfreq", C.c_int32), ("k0", C.POINTER(C.c_double)),
                ("src", C.POINTER(C.c_double)),
                ("nobj", C.c_int32), ("w", C.POINTER(C.c_double)),
                ("objective_kind", C.c_int32),
                ("obj_norm", C.POINTER(C.c_double)),
                ("pixel_kind", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("k_refresh", C.c_int32),
                ("k_fold", C.c_int32), ("max_accepts", C.c_int32),
                ("max_sweeps", C.c_int32), ("max_tile", C.c_int32),
                ("eta", C.c_double), ("guard", C.c_double), ("flags", C.c_uint64)]


class DbsResult(C.Structure):
    _fields_ = [("n_accepted", C.c_int32), ("sweeps", C.c_int32),
                ("converged", C.c_int32), ("n_refresh", C.c_int32),
                ("attempts", C.c_int64), ("n_verified", C.c_int64),
                ("f_initial", C.c_double), ("f_final", C.c_double)]


_lib = None

EXPORTS = {
    "pngf_version": ([], C.c_char_p),
    "pngf_last_error": ([C.c_void_p], C.c_char_p),
    "pngf_precompute": ([C.POINTER(Problem), C.POINTER(C.c_void_p)], C.c_int),
    "pngf_get_precompute": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p], C.c_int),
    "pngf_objective_norm": ([C.c_void_p, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "pngf_sizes": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "pngf_precompute_seconds": ([C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "pngf_workspace_bytes": ([C.c_void_p, C.POINTER(Options), C.POINTER(C.c_size_t)], C.c_int),
    "pngf_bind": ([C.c_void_p, C.POINTER(Options), C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "pngf_set_design": ([C.c_void_p, C.c_void_p], C.c_int),
    "pngf_evaluate": ([C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_void_p], C.c_int),
    "pngf_score_flips": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "pngf_gradient": ([C.c_void_p, C.c_void_p], C.c_int),
    "pngf_flip_set": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "pngf_tile_dbs_run": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                           C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pngf_accept_flips": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "pngf_refresh": ([C.c_void_p], C.c_int),
    "pngf_dbs_run": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                      C.POINTER(DbsResult)], C.c_int),
    "pngf_kernel_times": ([C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                           C.POINTER(C.c_int64)], C.c_int),
    "pngf_set_persist_spin": ([C.c_void_p, C.c_int32], C.c_int),
    "pngf_set_inverse_check": ([C.c_void_p, C.c_double], C.c_int),
    "pngf_inverse_stats": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "pngf_force_singular_refresh": ([C.c_void_p, C.c_int32], C.c_int),
    "pngf_destroy": ([C.c_void_p], C.c_int),
    "pngf_batch_create": ([C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)], C.c_int),
    "pngf_batch_last_error": ([C.c_void_p], C.c_char_p),
    "pngf_batch_workspace_bytes": ([C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "pngf_batch_bind": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "pngf_batch_set_grid": ([C.c_void_p, C.c_int32], C.c_int),
    "pngf_batch_dbs_run": ([C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(C.c_void_p),
                            C.POINTER(C.c_void_p), C.c_void_p, C.c_int32], C.c_int),
    "pngf_batch_tuning": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                           C.POINTER(C.c_int32)], C.c_int),
    "pngf_batch_ms_per_step": ([C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "pngf_batch_destroy": ([C.c_void_p], C.c_int),
    "pngf_model_create": ([C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)],
                          C.c_int),
    "pngf_model_last_error": ([C.c_void_p], C.c_char_p),
    "pngf_model_num_params": ([C.c_void_p, C.POINTER(C.c_int32)], C.c_int),
    "pngf_model_workspace_bytes": ([C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "pngf_model_bind": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "pngf_model_get_params": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "pngf_model_set_params": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "pngf_model_forward": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "pngf_model_forward_noalloc": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                    C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "pngf_model_train_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                               C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "pngf_model_destroy": ([C.c_void_p], C.c_int),
    "pngf_features": ([C.c_void_p, C.c_void_p], C.c_int),
    "pngf_learned_dbs_run": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                              C.c_void_p, C.POINTER(DbsResult)], C.c_int),
}


def lib():
    """Load libpngf.so (built in-tree); raise if it is missing.

    torch is imported first so that its HIP runtime is the one libpngf binds
    to (the dynamic linker matches libpngf's libamdhip64.so.7 dependency to the
    already-loaded copy by SONAME); two HIP runtimes in one process would not
    share devices, memory or streams.
    """
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the process-wide HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2501_18054_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _cplx(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def default_options(precision=PNGF_FP64_PLAIN, max_accepts=1 << 16, max_sweeps=32,
                    eta=1e-9, k_refresh=None, k_fold=0, guard=0.0, timing=False, max_tile=0,
                    step_launches=False, timing_steps=False, pivot_search=False):
    """Options of pngf_bind; k_refresh defaults to 32 for the mixed form and
    to 0 (no re-anchoring) for the others.  step_launches: one kernel launch
    per step of the mixed search instead of one launch per batch.  timing:
    events around every kernel class; timing_steps: around the step
    launches only.  pivot_search: every FP64 inversion with the pivot search
    (else without row exchanges first, checked)."""
    if k_refresh is None:
        k_refresh = 32 if precision == PNGF_MIXED else 0
    flags = ((PNGF_FLAG_TIMING if timing else 0) | (PNGF_FLAG_STEP_LAUNCHES if step_launches else 0)
             | (PNGF_FLAG_TIMING_STEPS if timing_steps else 0)
             | (PNGF_FLAG_PIVOT_SEARCH if pivot_search else 0))
    return Options(precision, k_refresh, k_fold, max_accepts, max_sweeps, max_tile, eta, guard,
                   flags)


class Handle:
    """One precomputed problem plus its device state (see include/pngf.h)."""

    def __init__(self, prob):
        L = lib()
        self._keep = dict(
            eps=np.ascontiguousarray(prob.eps_static, dtype=np.float64),
            mask=np.ascontiguousarray(prob.design_mask, dtype=np.uint8),
            k0=np.ascontiguousarray(prob.k0, dtype=np.float64),
            src=_cplx(prob.src), w=_cplx(prob.w),
            norm=np.ascontiguousarray(prob.obj_norm, dtype=np.float64))
        k = self._keep
        p = Problem(prob.nx, prob.ny, prob.npml, prob.h,
                    k["eps"].ctypes.data_as(C.POINTER(C.c_double)),
                    k["mask"].ctypes.data_as(C.POINTER(C.c_uint8)),
                    prob.eps_lo, prob.eps_hi, prob.nfreq,
                    k["k0"].ctypes.data_as(C.POINTER(C.c_double)),
                    k["src"].ctypes.data_as(C.POINTER(C.c_double)),
                    int(prob.w.shape[0]),
                    k["w"].ctypes.data_as(C.POINTER(C.c_double)),
                    int(prob.objective_kind),
                    k["norm"].ctypes.data_as(C.POINTER(C.c_double)),
                    int(getattr(prob, "pixel_kind", PNGF_PIXEL_DIELECTRIC)))
        h = C.c_void_p()
        rc = L.pngf_precompute(C.byref(p), C.byref(h))
        if rc != 0:
            raise PngfError(rc, L.pngf_last_error(None).decode())
        self._h = h
        nd, nf = C.c_int32(), C.c_int32()
        L.pngf_sizes(h, C.byref(nd), C.byref(nf))
        self.n_d, self.nfreq = nd.value, nf.value
        self._ws = None
        self._keep = None

    # ---------------------------------------------------------------- utils
    def _check(self, rc):
        if rc != 0:
            raise PngfError(rc, lib().pngf_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().pngf_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- precompute
    def precompute_seconds(self):
        s = C.c_double()
        self._check(lib().pngf_precompute_seconds(self._h, C.byref(s)))
        return s.value

    def get_precompute(self, fi=0):
        nd = self.n_d
        G = np.empty((nd, nd), np.complex128)
        b = np.empty(nd, np.complex128)
        god = np.empty(nd, np.complex128)
        xb = np.empty(1, np.complex128)
        self._check(lib().pngf_get_precompute(self._h, fi, _ptr(G), _ptr(b), _ptr(god), _ptr(xb)))
        return G, b, god, complex(xb[0])

    def objective_norm(self, fi=0):
        v = C.c_double()
        self._check(lib().pngf_objective_norm(self._h, fi, C.byref(v)))
        return v.value

    # --------------------------------------------------------------- device
    def workspace_bytes(self, opts):
        n = C.c_size_t()
        self._check(lib().pngf_workspace_bytes(self._h, C.byref(opts), C.byref(n)))
        return n.value

    def bind(self, opts=None, device="cuda:0", stream=None):
        """Allocate the workspace as a torch tensor and bind it with a stream."""
        import torch
        opts = opts or default_options()
        nbytes = self.workspace_bytes(opts)
        # the old workspace is released only after pngf_bind, which first waits
        # for work still queued on it (an initial inverse set_design left)
        old = self._ws
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(torch.device(device))
        self._stream = stream
        try:
            self._check(lib().pngf_bind(self._h, C.byref(opts), C.c_void_p(aligned),
                                        nbytes, C.c_void_p(stream.cuda_stream)))
        finally:
            del old
        self.opts = opts
        return self

    def set_design(self, bits):
        b = np.ascontiguousarray(bits, dtype=np.uint8)
        assert b.shape == (self.n_d,)
        self._check(lib().pngf_set_design(self._h, _ptr(b)))

    def evaluate(self, fields=False):
        f = C.c_double()
        x = np.empty(self.nfreq, np.complex128)
        e = np.empty((self.nfreq, self.n_d), np.complex128) if fields else None
        self._check(lib().pngf_evaluate(self._h, C.byref(f), _ptr(x), _ptr(e)))
        return (f.value, x, e) if fields else (f.value, x)

    def score_flips(self, cand):
        c = np.ascontiguousarray(cand, dtype=np.int32)
        out = np.empty(c.shape[0], np.float64)
        self._check(lib().pngf_score_flips(self._h, _ptr(c), c.shape[0], _ptr(out)))
        return out

    def gradient(self):
        """df/d eps_m for every pixel at the current design (pngf_gradient)."""
        out = np.empty(self.n_d, np.float64)
        self._check(lib().pngf_gradient(self._h, _ptr(out)))
        return out

    def flip_set(self, pix):
        """Flip the distinct pixels pix together (pngf_flip_set)."""
        p = np.ascontiguousarray(pix, dtype=np.int32)
        self._check(lib().pngf_flip_set(self._h, _ptr(p), p.shape[0]))

    def accept_flips(self, pix):
        p = np.ascontiguousarray(pix, dtype=np.int32)
        self._check(lib().pngf_accept_flips(self._h, _ptr(p), p.shape[0]))

    def refresh(self):
        self._check(lib().pngf_refresh(self._h))

    def dbs_run(self, perms):
        perms = np.ascontiguousarray(perms, dtype=np.int32)
        ns = perms.shape[0]
        cap = self.opts.max_accepts
        acc = np.empty(cap, np.int32)
        ftr = np.empty(cap, np.float64)
        res = DbsResult()
        self._check(lib().pngf_dbs_run(self._h, _ptr(perms), ns, _ptr(acc), _ptr(ftr),
                                       C.byref(res)))
        n = res.n_accepted
        return dict(accepted=acc[:n].copy(), f_trace=ftr[:n].copy(), n_accepted=n,
                    sweeps=res.sweeps, converged=bool(res.converged),
                    attempts=int(res.attempts), n_refresh=res.n_refresh,
                    n_verified=int(res.n_verified), f_initial=res.f_initial,
                    f_final=res.f_final)

    def tile_dbs_run(self, tiles, perms):
        """Search over tiles of pixels flipped together (pngf_tile_dbs_run):
        tiles (n_tiles, M) pixel ids, -1 padded; perms (n_sweeps, n_tiles)."""
        tiles = np.ascontiguousarray(tiles, dtype=np.int32)
        perms = np.ascontiguousarray(perms, dtype=np.int32)
        nt, m = tiles.shape
        cap = self.opts.max_accepts
        acc = np.empty(cap, np.int32)
        ftr = np.empty(cap, np.float64)
        res = DbsResult()
        self._check(lib().pngf_tile_dbs_run(self._h, _ptr(tiles), nt, m, _ptr(perms),
                                            perms.shape[0], _ptr(acc), _ptr(ftr),
                                            C.byref(res)))
        n = res.n_accepted
        return dict(accepted=acc[:n].copy(), f_trace=ftr[:n].copy(), n_accepted=n,
                    sweeps=res.sweeps, converged=bool(res.converged),
                    attempts=int(res.attempts), n_refresh=res.n_refresh,
                    f_initial=res.f_initial, f_final=res.f_final)

    def features(self):
        """CNN inputs of the current state, float32 [7, n_d]."""
        X = np.empty((Model.CHANNELS[0], self.n_d), np.float32)
        self._check(lib().pngf_features(self._h, _ptr(X)))
        return X

    def learned_dbs_run(self, model, k=64, max_accepts=None):
        """Ranked search (see pngf_learned_dbs_run): model None ranks by the
        first-order change; a Model must share this handle's stream."""
        cap = int(max_accepts if max_accepts is not None else self.opts.max_accepts)
        acc = np.empty(max(cap, 1), np.int32)
        ftr = np.empty(max(cap, 1), np.float64)
        res = DbsResult()
        mp = model._m if model is not None else None
        self._check(lib().pngf_learned_dbs_run(self._h, mp, int(k), cap, _ptr(acc),
                                               _ptr(ftr), C.byref(res)))
        n = res.n_accepted
        return dict(accepted=acc[:n].copy(), f_trace=ftr[:n].copy(), n_accepted=n,
                    extra_chunks=res.sweeps, converged=bool(res.converged),
                    attempts=int(res.attempts), f_initial=res.f_initial, f_final=res.f_final)

    def force_singular_refresh(self, n):
        """Test hook: the next n block-Woodbury refreshes report singular."""
        self._check(lib().pngf_force_singular_refresh(self._h, int(n)))

    def set_inverse_check(self, tol):
        """Probe-residual bound of the inversion without row exchanges."""
        self._check(lib().pngf_set_inverse_check(self._h, float(tol)))

    def inverse_stats(self):
        """(inversions without row exchanges, inversions with the pivot search)."""
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().pngf_inverse_stats(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_persist_spin(self, polls):
        """Bound of a persistent-search grid-barrier wait, in polls."""
        self._check(lib().pngf_set_persist_spin(self._h, int(polls)))

    def kernel_times(self, name):
        t = C.c_double()
        n = C.c_int64()
        self._check(lib().pngf_kernel_times(self._h, KERNEL_IDS[name], C.byref(t), C.byref(n)))
        return t.value, n.value


class Batch:
    """Many handles advanced together (see the batch section of pngf.h)."""

    def __init__(self, handles, stream=None):
        import torch
        L = lib()
        self.handles = list(handles)
        arr = (C.c_void_p * len(self.handles))(*[h._h for h in self.handles])
        b = C.c_void_p()
        rc = L.pngf_batch_create(arr, len(self.handles), C.byref(b))
        if rc != 0:
            raise PngfError(rc, L.pngf_batch_last_error(None).decode())
        self._b = b
        n = C.c_size_t()
        self._check(L.pngf_batch_workspace_bytes(b, C.byref(n)))
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device="cuda:0")
        aligned = (self._ws.data_ptr() + 255) & ~255
        stream = stream or self.handles[0]._stream
        self._check(L.pngf_batch_bind(b, C.c_void_p(aligned), n.value,
                                      C.c_void_p(stream.cuda_stream)))

    def _check(self, rc):
        if rc != 0:
            raise PngfError(rc, lib().pngf_batch_last_error(self._b).decode())

    def set_grid(self, grid):
        self._check(lib().pngf_batch_set_grid(self._b, int(grid)))

    def dbs_run(self, perms, autotune=False):
        n = len(self.handles)
        ps = [np.ascontiguousarray(p, dtype=np.int32) for p in perms]
        ns = np.array([p.shape[0] for p in ps], dtype=np.int32)
        accs = [np.empty(h.opts.max_accepts, np.int32) for h in self.handles]
        ftrs = [np.empty(h.opts.max_accepts, np.float64) for h in self.handles]
        res = (DbsResult * n)()
        pp = (C.c_void_p * n)(*[p.ctypes.data for p in ps])
        ap = (C.c_void_p * n)(*[a.ctypes.data for a in accs])
        fp = (C.c_void_p * n)(*[f.ctypes.data for f in ftrs])
        self._check(lib().pngf_batch_dbs_run(self._b, pp, _ptr(ns), ap, fp, C.byref(res),
                                             1 if autotune else 0))
        out = []
        for k in range(n):
            r = res[k]
            m = r.n_accepted
            out.append(dict(accepted=accs[k][:m].copy(), f_trace=ftrs[k][:m].copy(),
                            n_accepted=m, sweeps=r.sweeps, converged=bool(r.converged),
                            attempts=int(r.attempts), n_refresh=r.n_refresh,
                            n_verified=int(r.n_verified), f_initial=r.f_initial,
                            f_final=r.f_final))
        return out

    def tuning(self):
        """[(grid, rows per work item, device ms per step)] of the shapes tried."""
        g = np.empty(32, np.int32)
        rows = np.empty(32, np.int32)
        ms = np.empty(32, np.float64)
        n = C.c_int32()
        self._check(lib().pngf_batch_tuning(self._b, _ptr(g), _ptr(rows), _ptr(ms), 32,
                                            C.byref(n)))
        k = n.value
        return list(zip(g[:k].tolist(), rows[:k].tolist(), ms[:k].tolist()))

    def ms_per_step(self):
        v = C.c_double()
        self._check(lib().pngf_batch_ms_per_step(self._b, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_b", None):
            lib().pngf_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def model_forward_noalloc(params, X, Y, stream=None):
    """pngf_model_forward_noalloc on device tensors: params (float32, flat),
    X (float32 [N, 7, H, W]) in, Y (float32 [N, 1, H, W]) out; queued on
    stream (torch's current one by default)."""
    import torch
    for t in (params, X, Y):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    N, c, H, W = X.shape
    assert c == Model.CHANNELS[0] and tuple(Y.shape) == (N, 1, H, W)
    if stream is None:
        stream = torch.cuda.current_stream(X.device)
    rc = lib().pngf_model_forward_noalloc(C.c_void_p(params.data_ptr()), int(params.numel()),
                                          C.c_void_p(X.data_ptr()), int(N), int(H), int(W),
                                          C.c_void_p(Y.data_ptr()), C.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise PngfError(rc, lib().pngf_model_last_error(None).decode())


class Model:
    """Flip-proposal CNN of libpngf (see the learned section of pngf.h).

    Parameters are flat float32 [W1, b1, ..., W4, b4], W as [out][in][3][3].
    """

    CHANNELS = (7, 32, 32, 32, 1)

    def __init__(self, H, W, max_batch=64, seed=0, device="cuda:0", stream=None):
        import torch
        L = lib()
        m = C.c_void_p()
        rc = L.pngf_model_create(int(H), int(W), int(max_batch), int(seed), C.byref(m))
        if rc != 0:
            raise PngfError(rc, L.pngf_model_last_error(None).decode())
        self._m = m
        self.H, self.W, self.max_batch = int(H), int(W), int(max_batch)
        n = C.c_int32()
        self._check(L.pngf_model_num_params(m, C.byref(n)))
        self.num_params = n.value
        nb = C.c_size_t()
        self._check(L.pngf_model_workspace_bytes(m, C.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=device)
        aligned = (self._ws.data_ptr() + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(torch.device(device))
        self._stream = stream
        self._check(L.pngf_model_bind(m, C.c_void_p(aligned), nb.value,
                                      C.c_void_p(stream.cuda_stream)))

    def _check(self, rc):
        if rc != 0:
            raise PngfError(rc, lib().pngf_model_last_error(self._m).decode())

    def shapes(self):
        ch = self.CHANNELS
        out = []
        for cin, cout in zip(ch[:-1], ch[1:]):
            out += [(cout, cin, 3, 3), (cout,)]
        return out

    def unflatten(self, flat):
        out, o = [], 0
        for s in self.shapes():
            n = int(np.prod(s))
            out.append(np.asarray(flat[o:o + n]).reshape(s))
            o += n
        return out

    def get_params(self):
        p = np.empty(self.num_params, np.float32)
        self._check(lib().pngf_model_get_params(self._m, _ptr(p), self.num_params))
        return p

    def set_params(self, flat):
        p = np.ascontiguousarray(flat, dtype=np.float32)
        assert p.shape == (self.num_params,)
        self._check(lib().pngf_model_set_params(self._m, _ptr(p), self.num_params))

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        N = X.shape[0]
        assert X.shape == (N, self.CHANNELS[0], self.H, self.W)
        Y = np.empty((N, 1, self.H, self.W), np.float32)
        self._check(lib().pngf_model_forward(self._m, _ptr(X), N, _ptr(Y)))
        return Y

    def train_step(self, X, T, lr=1e-3, want_grads=False):
        """One forward/backward (+ Adam if lr > 0); returns (loss, grads)."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        N = X.shape[0]
        assert X.shape == (N, self.CHANNELS[0], self.H, self.W)
        assert T.shape == (N, 1, self.H, self.W)
        g = np.empty(self.num_params, np.float32) if want_grads else None
        loss = C.c_double()
        self._check(lib().pngf_model_train_step(self._m, _ptr(X), _ptr(T), N, float(lr),
                                                C.byref(loss), _ptr(g)))
        return loss.value, g

    def close(self):
        if getattr(self, "_m", None):
            lib().pngf_model_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
