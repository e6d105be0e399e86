"""ctypes binding of libsdmm.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module converts
problem dicts into the C structure, torch device tensors into pointers and
the results back into numpy arrays.  It fails loudly when the library is not
built or no GPU is present.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdmm.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, ESTATE, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
PREC = {"fp64": 0, "mixed": 1}
METHOD = {"stochastic": 0, "deterministic": 1, "per_iteration": 2}
FIELDS = {"lambda": 0, "darcy_p": 1, "darcy_u": 2, "stokes_u": 3, "stokes_p": 4}
MAPS = {"interfaces": 0, "sub_ptr": 1, "sub_dofs": 2, "sub_sign": 3, "g2l": 4, "nlocal": 5, "node_ids": 6}

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


class CProblem(ctypes.Structure):
    _fields_ = [("nu_s", ctypes.c_double), ("nu_d", ctypes.c_double), ("alpha", ctypes.c_double),
                ("k_bjs", ctypes.c_double), ("inflow_x", ctypes.c_double), ("inflow_y", ctypes.c_double),
                ("inflow_shear", ctypes.c_double), ("p_bottom", ctypes.c_double), ("domain", ctypes.c_double * 4),
                ("n_sub", ctypes.c_int32), ("sub_type", _i32p), ("sub_rect", _f64p), ("sub_n", _i32p),
                ("sub_region", _i32p), ("mortar_degree", ctypes.c_int32), ("mortar_elements", ctypes.c_int32),
                ("n_region", ctypes.c_int32), ("region_rect", _f64p), ("region_nterm", _i32p),
                ("region_sigma2", _f64p), ("region_eta", _f64p), ("region_mean_logk", _f64p),
                ("rule_kind", ctypes.c_int32), ("rule_m", ctypes.c_int32), ("rule_level", ctypes.c_int32),
                ("rule_growth", ctypes.c_int32), ("stokes_element", ctypes.c_int32), ("darcy_mass", ctypes.c_int32)]


class CSizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_sub", "n_stokes", "n_darcy", "n_iface", "M", "n_real", "n_term",
                                              "n_region", "n_units", "n_floating", "n_kernel")] + \
               [("field_size", ctypes.c_int64 * 5)] + \
               [(n, ctypes.c_int64) for n in ("basis_bytes", "response_bytes", "max_R", "darcy_flops")]


class CCounters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("basis_solves_darcy", "basis_solves_stokes", "complementary_solves",
                                              "units_built", "refinement_steps", "cg_iterations", "realizations")] + \
               [(n, ctypes.c_double) for n in ("ms_basis_darcy", "ms_basis_stokes", "ms_solve", "max_refine_residual")] + \
               [(n, ctypes.c_int64) for n in ("cg_launches", "cg_timed_launches", "cg_timed_active", "cg_timed_columns")] + \
               [(n, ctypes.c_double) for n in ("ms_cg_apply", "ms_cg_update", "ms_moments", "ms_basis_build")]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)


class CAlloc(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("user", ctypes.c_void_p)]


_vp, _i64, _i32, _f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
EXPORTS = {
    "sdmm_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(CAlloc), ctypes.POINTER(_vp)]),
    "sdmm_destroy": (ctypes.c_int, [_vp]),
    "sdmm_last_error": (ctypes.c_char_p, [_vp]),
    "sdmm_set_problem": (ctypes.c_int, [_vp, ctypes.POINTER(CProblem), _i64p]),
    "sdmm_release_problem": (ctypes.c_int, [_vp, _i64]),
    "sdmm_get_sizes": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(CSizes)]),
    "sdmm_get_index_maps": (ctypes.c_int, [_vp, _i64, ctypes.c_int, _i64p, _i64, _i64p]),
    "sdmm_get_collocation": (ctypes.c_int, [_vp, _i64, _f64p, _f64p]),
    "sdmm_get_kl": (ctypes.c_int, [_vp, _i64, ctypes.c_int, _f64p, _i32p]),
    "sdmm_build_flux_basis": (ctypes.c_int, [_vp, _i64, ctypes.c_int, ctypes.c_int, _vp]),
    "sdmm_get_basis": (ctypes.c_int, [_vp, _i64, ctypes.c_int, ctypes.c_int, _f64p, _i64]),
    "sdmm_solve_interface": (ctypes.c_int, [_vp, _i64, _i64, _vp, _vp, _f64, _i32, _vp, _vp, _vp, _vp, _vp]),
    "sdmm_solve_interface_noalloc": (ctypes.c_int, [_vp, _i64, _i64, _vp, _f64, _i32, _vp, _vp, _vp, _vp, _vp]),
    "sdmm_noalloc_scratch_bytes": (ctypes.c_int, [_i64p]),
    "sdmm_stream_open": (ctypes.c_int, [_vp, _i64, _i64, _f64, _i32, _vp, _i64p]),
    "sdmm_stream_submit": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64p, _vp, _vp, _vp, _vp, _i64p]),
    "sdmm_stream_run": (ctypes.c_int, [_vp, _i64, _i64, _i32, _i64p, _i64, _i64p, _i64p]),
    "sdmm_stream_close": (ctypes.c_int, [_vp, _i64, _i64]),
    "sdmm_get_interface_data": (ctypes.c_int, [_vp, _i64, _f64p, _f64p]),
    "sdmm_autotune": (ctypes.c_int, [_vp, _i64, _i64, _vp, _f64, _i32, _vp, _i64p]),
    "sdmm_accumulate_moments": (ctypes.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp]),
    "sdmm_get_moments": (ctypes.c_int, [_vp, _i64, ctypes.c_int, _f64p, _f64p, _i64]),
    "sdmm_reset_moments": (ctypes.c_int, [_vp, _i64]),
    "sdmm_finalize_moments": (ctypes.c_int, [_vp, _i64, _vp]),
    "sdmm_get_counters": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(CCounters)]),
    "sdmm_set_option": (ctypes.c_int, [_vp, _i64, ctypes.c_int, _i64]),
}
OPTIONS = {"cg_chunk": 0, "cg_check": 1, "cg_graph": 2, "kernel_timing": 3, "cg_lanes": 4, "stokes_rebuild": 5, "stokes_refine": 6,
           "basis_launch": 7}

_LIB = None


def load():
    """Load libsdmm.so and declare its signatures (no GPU call is made)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsdmm.so is not built; run paper_1802_06263_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


class SdmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sdmm error %d: %s" % (code, msg))
        self.code = code


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dptr(t):
    """Device pointer of a torch tensor (must live on the GPU)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _torch_allocator():
    """sdmm_alloc callbacks backed by torch's caching allocator."""
    import torch

    def alloc(nbytes, device, user):
        try:
            with torch.cuda.device(device):
                return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:
            return None

    def release(ptr, nbytes, device, user):
        torch.cuda.caching_allocator_delete(ptr)

    fa, fr = _ALLOC_FN(alloc), _RELEASE_FN(release)
    return CAlloc(fa, fr, None), (fa, fr)


class Context:
    """One library context on one GPU.  A context holds any number of
    problems; set_problem() makes the new problem the default one, and every
    method takes an optional problem id `pid` instead."""

    def __init__(self, device=0, torch_alloc=False):
        if device >= 0:
            # torch brings its own HIP runtime; it must be initialised before the
            # library's first HIP call, or torch no longer sees the device
            import torch
            torch.cuda.init()
        self.lib = load()
        h = ctypes.c_void_p()
        self._alloc_keep = None
        al = None
        if torch_alloc:
            cal, self._alloc_keep = _torch_allocator()
            self._alloc_struct = cal
            al = ctypes.byref(cal)
        rc = self.lib.sdmm_create(int(device), al, ctypes.byref(h))
        if rc != OK:
            raise SdmmError(rc, "sdmm_create failed (no usable GPU %d?)" % device)
        self.h = h
        self.pid = None
        self._sz = {}

    def close(self):
        if self.h:
            self.lib.sdmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise SdmmError(rc, self.lib.sdmm_last_error(self.h).decode())
        return rc

    def _id(self, pid):
        pid = self.pid if pid is None else pid
        if pid is None:
            raise SdmmError(ESTATE, "no problem set")
        return ctypes.c_int64(pid)

    @property
    def _sizes(self):
        return self._sz[self.pid]

    # ---- problem -------------------------------------------------------------
    def set_problem(self, prob):
        """Add a problem; it becomes the default one.  Returns its id."""
        subs = prob["subdomains"]
        ph = prob["physics"]
        regs = prob["regions"]
        rule = prob["rule"]
        keep = {
            "sub_type": _arr([0 if s["type"] == "stokes" else 1 for s in subs], np.int32),
            "sub_rect": _arr([s["rect"] for s in subs], np.float64),
            "sub_n": _arr([s["n"] for s in subs], np.int32),
            "sub_region": _arr([s["region"] if s["type"] == "darcy" else -1 for s in subs], np.int32),
            "region_rect": _arr([r["rect"] for r in regs], np.float64),
            "region_nterm": _arr([r["nterm"] for r in regs], np.int32),
            "region_sigma2": _arr([r["sigma2"] for r in regs], np.float64),
            "region_eta": _arr([r["eta"] for r in regs], np.float64),
            "region_mean_logk": _arr([r["mean_logk"] for r in regs], np.float64),
        }
        c = CProblem()
        c.nu_s, c.nu_d, c.alpha, c.k_bjs = ph["nu_s"], ph["nu_d"], ph["alpha"], ph["k_bjs"]
        c.inflow_x, c.inflow_y = ph["inflow"]
        c.inflow_shear = float(ph.get("inflow_shear", 0.0))
        c.p_bottom = ph["p_bottom"]
        for k in range(4):
            c.domain[k] = prob["domain"][k]
        c.n_sub = len(subs)
        c.sub_type = _ptr(keep["sub_type"], ctypes.c_int32)
        c.sub_rect = _ptr(keep["sub_rect"], ctypes.c_double)
        c.sub_n = _ptr(keep["sub_n"], ctypes.c_int32)
        c.sub_region = _ptr(keep["sub_region"], ctypes.c_int32)
        c.mortar_degree = prob["mortar"]["degree"]
        c.mortar_elements = prob["mortar"]["elements"]
        c.n_region = len(regs)
        c.region_rect = _ptr(keep["region_rect"], ctypes.c_double)
        c.region_nterm = _ptr(keep["region_nterm"], ctypes.c_int32)
        c.region_sigma2 = _ptr(keep["region_sigma2"], ctypes.c_double)
        c.region_eta = _ptr(keep["region_eta"], ctypes.c_double)
        c.region_mean_logk = _ptr(keep["region_mean_logk"], ctypes.c_double)
        c.rule_kind = 0 if rule["kind"] == "tensor" else 1
        c.rule_m = int(rule.get("m", 0))
        c.rule_level = int(rule.get("level", 0))
        c.rule_growth = 0 if rule.get("growth", "paper") == "paper" else 1
        disc = prob.get("discretization", {})
        c.stokes_element = {"q2q1": 0, "p2p1": 1}[disc.get("stokes", "q2q1")]
        c.darcy_mass = {"trapezoidal": 0, "exact": 1}[disc.get("darcy", "trapezoidal")]
        pid = ctypes.c_int64()
        self._check(self.lib.sdmm_set_problem(self.h, ctypes.byref(c), ctypes.byref(pid)))
        self.pid = pid.value
        self._sz[self.pid] = self.sizes()
        return self.pid

    def release_problem(self, pid):
        self._check(self.lib.sdmm_release_problem(self.h, ctypes.c_int64(pid)))
        self._sz.pop(pid, None)
        if self.pid == pid:
            self.pid = None

    def sizes(self, pid=None):
        s = CSizes()
        self._check(self.lib.sdmm_get_sizes(self.h, self._id(pid), ctypes.byref(s)))
        out = {n: getattr(s, n) for n, _ in CSizes._fields_ if n != "field_size"}
        out["field_size"] = [s.field_size[k] for k in range(5)]
        return out

    def index_map(self, kind, pid=None):
        n = ctypes.c_int64()
        k = MAPS[kind]
        self._check(self.lib.sdmm_get_index_maps(self.h, self._id(pid), k, None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int64)
        self._check(self.lib.sdmm_get_index_maps(self.h, self._id(pid), k, _ptr(out, ctypes.c_int64), out.size,
                                                 ctypes.byref(n)))
        return out[:n.value]

    def collocation(self, pid=None):
        s = self._sz[self._id(pid).value]
        pts = np.zeros((s["n_real"], max(s["n_term"], 1)))
        w = np.zeros(s["n_real"])
        self._check(self.lib.sdmm_get_collocation(self.h, self._id(pid), _ptr(pts, ctypes.c_double),
                                                  _ptr(w, ctypes.c_double)))
        return pts[:, :s["n_term"]], w

    def kl(self, region, nterm, pid=None):
        lam = np.zeros(nterm)
        modes = np.zeros(2 * nterm, dtype=np.int32)
        self._check(self.lib.sdmm_get_kl(self.h, self._id(pid), region, _ptr(lam, ctypes.c_double),
                                         _ptr(modes, ctypes.c_int32)))
        return lam, modes.reshape(nterm, 2)

    # ---- hot path --------------------------------------------------------------
    def build_flux_basis(self, precision="fp64", method="stochastic", stream=None, pid=None, allow_notconv=False):
        rc = self.lib.sdmm_build_flux_basis(self.h, self._id(pid), METHOD[method], PREC[precision], _stream(stream))
        return self._check(rc, allow=(ENOTCONV,) if allow_notconv else ())

    def get_basis(self, sub, k, R, pid=None):
        S = np.zeros((R, R), order="F")
        self._check(self.lib.sdmm_get_basis(self.h, self._id(pid), sub, k, _ptr(S, ctypes.c_double), R))
        return S

    def solve_interface(self, gidx, lam, rtol=1e-8, max_iter=None, iters=None, relres=None, status=None,
                        stream=None, allow_notconv=False, pid=None, y=None):
        """gidx: int64 device tensor (n), or None with y: float64 device tensor
        (n x n_term) of off-grid points; lam: float64 device tensor (n x M)."""
        n = gidx.numel() if gidx is not None else y.shape[0]
        sz = self._sz[self._id(pid).value]
        if max_iter is None:
            max_iter = 10 * sz["M"]
        rc = self.lib.sdmm_solve_interface(self.h, self._id(pid), n, _dptr(gidx), _dptr(y), float(rtol),
                                           int(max_iter), _dptr(lam), _dptr(iters), _dptr(relres), _dptr(status),
                                           _stream(stream))
        return self._check(rc, allow=(ENOTCONV,) if allow_notconv else ())

    def solve_interface_noalloc(self, gidx, lam, rtol=1e-8, max_iter=None, iters=None, relres=None,
                                status=None, stream=None, allow_notconv=False, pid=None):
        """sdmm_solve_interface_noalloc: the same solve with the CG workspace in
        the library's fixed per-GPU scratch array (no device allocation)."""
        sz = self._sz[self._id(pid).value]
        if max_iter is None:
            max_iter = 10 * sz["M"]
        rc = self.lib.sdmm_solve_interface_noalloc(self.h, self._id(pid), gidx.numel(), _dptr(gidx), float(rtol),
                                                   int(max_iter), _dptr(lam), _dptr(iters), _dptr(relres),
                                                   _dptr(status), _stream(stream))
        return self._check(rc, allow=(ENOTCONV,) if allow_notconv else ())

    def noalloc_scratch_bytes(self):
        out = ctypes.c_int64()
        self._check(self.lib.sdmm_noalloc_scratch_bytes(ctypes.byref(out)))
        return out.value

    # ---- CG streams (continuous batching) -------------------------------------
    def stream_open(self, slots, rtol=1e-8, max_iter=None, stream=None, pid=None):
        sz = self._sz[self._id(pid).value]
        if max_iter is None:
            max_iter = 10 * sz["M"]
        sid = ctypes.c_int64()
        self._check(self.lib.sdmm_stream_open(self.h, self._id(pid), int(slots), float(rtol), int(max_iter),
                                              _stream(stream), ctypes.byref(sid)))
        return sid.value

    def stream_submit(self, sid, gidx, lam, iters=None, relres=None, status=None, pid=None):
        """gidx: host int64 array; lam (n x M) and the optional outputs: device tensors."""
        g = _arr(gidx, np.int64)
        t = ctypes.c_int64()
        self._check(self.lib.sdmm_stream_submit(self.h, self._id(pid), sid, g.size, _ptr(g, ctypes.c_int64),
                                                _dptr(lam), _dptr(iters), _dptr(relres), _dptr(status),
                                                ctypes.byref(t)))
        return t.value

    def stream_run(self, sid, max_groups=1, pid=None, cap=4096):
        """Advance the stream; returns (completed tickets, realizations in flight or queued)."""
        done = np.zeros(cap, dtype=np.int64)
        nd = ctypes.c_int64()
        fl = ctypes.c_int64()
        self._check(self.lib.sdmm_stream_run(self.h, self._id(pid), sid, int(max_groups), _ptr(done, ctypes.c_int64),
                                             cap, ctypes.byref(nd), ctypes.byref(fl)))
        return done[:nd.value].tolist(), fl.value

    def stream_close(self, sid, pid=None):
        self._check(self.lib.sdmm_stream_close(self.h, self._id(pid), sid))

    def interface_data(self, pid=None):
        """(g_H [M], G [n_kernel x M]) as host arrays."""
        sz = self._sz[self._id(pid).value]
        M, nk = sz["M"], sz["n_kernel"]
        g = np.zeros(M)
        G = np.zeros((max(nk, 1), M))
        self._check(self.lib.sdmm_get_interface_data(self.h, self._id(pid), _ptr(g, ctypes.c_double),
                                                     _ptr(G, ctypes.c_double)))
        return g, G[:nk]

    def autotune(self, gidx, rtol=1e-8, max_iter=None, stream=None, pid=None):
        """Pick the CG slot count (realizations in flight) on gidx (int64 device
        tensor); sets it as the cg_chunk option and returns it."""
        out = ctypes.c_int64()
        sz = self._sz[self._id(pid).value]
        if max_iter is None:
            max_iter = 10 * sz["M"]
        self._check(self.lib.sdmm_autotune(self.h, self._id(pid), gidx.numel(), _dptr(gidx), float(rtol),
                                           int(max_iter), _stream(stream), ctypes.byref(out)))
        return out.value

    def accumulate_moments(self, gidx, lam, weights=None, stream=None, pid=None, y=None):
        n = gidx.numel() if gidx is not None else y.shape[0]
        self._check(self.lib.sdmm_accumulate_moments(self.h, self._id(pid), n, _dptr(gidx), _dptr(y), _dptr(lam),
                                                     _dptr(weights), _stream(stream)))

    def get_moments(self, field, pid=None):
        n = self._sz[self._id(pid).value]["field_size"][FIELDS[field]]
        mean = np.zeros(max(n, 1))
        var = np.zeros(max(n, 1))
        self._check(self.lib.sdmm_get_moments(self.h, self._id(pid), FIELDS[field], _ptr(mean, ctypes.c_double),
                                              _ptr(var, ctypes.c_double), mean.size))
        return mean[:n], var[:n]

    def finalize_moments(self, stream=None, pid=None):
        self._check(self.lib.sdmm_finalize_moments(self.h, self._id(pid), _stream(stream)))

    def reset_moments(self, pid=None):
        self._check(self.lib.sdmm_reset_moments(self.h, self._id(pid)))

    def set_option(self, name, value, pid=None):
        self._check(self.lib.sdmm_set_option(self.h, self._id(pid), OPTIONS[name], int(value)))

    def counters(self, pid=None):
        c = CCounters()
        self._check(self.lib.sdmm_get_counters(self.h, self._id(pid), ctypes.byref(c)))
        return {n: getattr(c, n) for n, _ in CCounters._fields_}
