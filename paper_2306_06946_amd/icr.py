"""ctypes binding of the C ABI in include/icr.h (argument marshalling only).

Device arguments are torch CUDA (HIP) tensors; their ``data_ptr()`` is passed
as a plain pointer and the scene runs on torch's current stream unless
another stream is given.  Every computation happens in ``libicr.so``; if the
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libicr.so")

OK, WARN_NOT_CONVERGED = 0, 1
FP64, FP32_IR = 0, 1
E_ARG, E_NOT_SPD, E_OOM, E_HIP, E_STATE = -1, -2, -3, -4, -5
SEPARATE, STICK, SLIP = 0, 1, 2


class IcrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"icr error {code}: {msg}")
        self.code = code


class Obstacle(C.Structure):
    _fields_ = [("kind", C.c_int32), ("c0", C.c_double * 3), ("vel", C.c_double * 3),
                ("normal", C.c_double * 3), ("radius", C.c_double)]


class StepOpts(C.Structure):
    _fields_ = [("n_contacts", C.c_int32), ("n_newton", C.c_int32), ("max_sweeps", C.c_int32),
                ("j_inner", C.c_int32), ("tol", C.c_double), ("timing", C.c_int32), ("scheme", C.c_int32),
                ("graph", C.c_int32), ("precision", C.c_int32), ("refine", C.c_int32)]


class StepReport(C.Structure):
    _fields_ = [("t", C.c_double), ("ms_total", C.c_double), ("ms_free", C.c_double),
                ("ms_contacts", C.c_double), ("ms_build_WH", C.c_double), ("ms_newton", C.c_double),
                ("ms_update_W", C.c_double), ("ms_pgs", C.c_double), ("ms_correct", C.c_double),
                ("sweeps", C.c_int32 * 16), ("eps", C.c_double * 16),
                ("n_separate", C.c_int32), ("n_stick", C.c_int32), ("n_slip", C.c_int32), ("ms_corr", C.c_double)]


class FactorInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_supernodes", C.c_int64), ("n_levels", C.c_int64), ("nnz_L", C.c_int64),
                ("max_front", C.c_int64), ("factor_flops", C.c_double), ("factor_ms", C.c_double),
                ("device_bytes", C.c_int64)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("scene", C.c_int32), ("status", C.c_int32), ("latency_ms", C.c_double),
                ("queue_ms", C.c_double)]


_P = C.c_void_p
_I = C.c_int32
_D = C.c_double

_SIGS = {
    "icr_create": (C.c_int, [C.POINTER(_P), _P]),
    "icr_destroy": (None, [_P]),
    "icr_last_error": (C.c_char_p, [_P]),
    "icr_set_stream": (C.c_int, [_P, _P]),
    "icr_set_overlap": (C.c_int, [_P, C.c_int32]),
    "icr_assemble": (C.c_int, [_P, _P, _I, _P, _I, _P, _P, _D, _D, _D, _D, _P, _P]),
    "icr_factor": (C.c_int, [_P]),
    "icr_get_factor_info": (C.c_int, [_P, C.POINTER(FactorInfo)]),
    "icr_build_WH": (C.c_int, [_P, _I, _P, _P, _P]),
    "icr_update_W": (C.c_int, [_P, _I, _P, _P, _P]),
    "icr_solve_contacts": (C.c_int, [_P, _I, _P, _P, _P, _D, _P, _P, _I, _D, _I, C.POINTER(_I),
                                     C.POINTER(_D)]),
    "icr_solve_contacts_noalloc": (C.c_int, [_P, _I, _P, _P, _P, _D, _P, _P, _I, _D, _I, C.POINTER(_I),
                                             C.POINTER(_D)]),
    "icr_proximity_update": (C.c_int, [_P, _I, _P, _P, _P, _D, _P]),
    "icr_set_candidates": (C.c_int, [_P, _I, _P, _P]),
    "icr_set_pairs": (C.c_int, [_P, _I, _P, _P, _P, _P]),
    "icr_step": (C.c_int, [_P, C.POINTER(Obstacle), C.POINTER(StepOpts), C.POINTER(StepReport)]),
    "icr_reserve": (C.c_int, [_P, _I, _I]),
    "icr_get_state": (C.c_int, [_P, _P, _P, C.POINTER(_D)]),
    "icr_set_state": (C.c_int, [_P, _P, _P, _D]),
    "icr_get_step_results": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "icr_analyze": (C.c_int, [_P, _I, _P, _I, _P, _P, _I, _P, _P, _I, C.POINTER(_I), C.POINTER(_I)]),
    "icr_server_create": (C.c_int, [C.POINTER(_P), C.c_int64, _I]),
    "icr_server_destroy": (None, [_P]),
    "icr_server_last_error": (C.c_char_p, [_P]),
    "icr_server_set_batching": (C.c_int, [_P, _I, C.c_double]),
    "icr_server_admit": (C.c_int, [_P, _P, C.POINTER(_I)]),
    "icr_server_evict": (C.c_int, [_P, _I]),
    "icr_server_used": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "icr_server_submit": (C.c_int, [_P, _I, C.POINTER(Obstacle), C.POINTER(StepOpts), C.c_uint64]),
    "icr_server_poll": (C.c_int, [_P, C.POINTER(Completion), _I, C.POINTER(_I), _I, C.POINTER(_I)]),
}

_lib = None


def lib():
    """Load libicr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_06946_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t, dtype=None, numel=None):
    """Pointer of a contiguous CUDA tensor (checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor has {t.numel()} elements, need {numel}")
    return C.c_void_p(t.data_ptr())


def analyze(nodes, tets):
    """Host-only nested dissection + supernodal structure (no GPU needed)."""
    L = lib()
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    N, T = len(nodes), len(tets)
    perm = np.zeros(N, dtype=np.int32)
    nsup, nrows = C.c_int32(0), C.c_int32(0)
    st = L.icr_analyze(_np_ptr(nodes), N, _np_ptr(tets), T, _np_ptr(perm), None, 0, None, None, 0,
                       C.byref(nsup), C.byref(nrows))
    if st != OK:
        raise IcrError(st, "icr_analyze failed")
    sup = np.zeros(4 * nsup.value, dtype=np.int32)
    rows_ptr = np.zeros(nsup.value + 1, dtype=np.int32)
    rows = np.zeros(max(1, nrows.value), dtype=np.int32)
    st = L.icr_analyze(_np_ptr(nodes), N, _np_ptr(tets), T, _np_ptr(perm), _np_ptr(sup), nsup.value,
                       _np_ptr(rows_ptr), _np_ptr(rows), len(rows), C.byref(nsup), C.byref(nrows))
    if st != OK:
        raise IcrError(st, "icr_analyze failed")
    return dict(perm=perm, sup=sup.reshape(-1, 4), rows_ptr=rows_ptr, rows=rows[:nrows.value])


class Scene:
    """One simulation scene on the current GPU (wraps an icr_scene handle)."""

    def __init__(self, stream=None):
        import torch
        self._torch = torch
        self.L = lib()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._h = C.c_void_p()
        st = self.L.icr_create(C.byref(self._h), C.c_void_p(stream))
        if st != OK:
            raise IcrError(st, "icr_create failed")
        self.n = 0
        self.N = 0

    def close(self):
        if self._h:
            self.L.icr_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow_warn=False):
        if st == OK or (allow_warn and st == WARN_NOT_CONVERGED):
            return st
        raise IcrError(st, self.L.icr_last_error(self._h).decode())

    def set_stream(self, stream):
        self._check(self.L.icr_set_stream(self._h, C.c_void_p(stream)))

    def set_overlap(self, enable):
        self._check(self.L.icr_set_overlap(self._h, 1 if enable else 0))

    # -- model ---------------------------------------------------------------
    def assemble(self, scene):
        nodes = np.ascontiguousarray(scene["nodes"], dtype=np.float64)
        tets = np.ascontiguousarray(scene["tets"], dtype=np.int32)
        E = np.ascontiguousarray(scene["E"], dtype=np.float64)
        nu = np.ascontiguousarray(scene["nu_e"], dtype=np.float64)
        g = np.ascontiguousarray(scene["gravity"], dtype=np.float64)
        fixed = np.ascontiguousarray(scene["fixed"], dtype=np.uint8)
        self._check(self.L.icr_assemble(self._h, _np_ptr(nodes), len(nodes), _np_ptr(tets), len(tets), _np_ptr(E),
                                        _np_ptr(nu), scene["rho"], scene["alpha"], scene["beta"], scene["h"],
                                        _np_ptr(g), _np_ptr(fixed)))
        self.N = len(nodes)
        self.n = 3 * self.N

    def factor(self):
        self._check(self.L.icr_factor(self._h))

    def factor_info(self):
        info = FactorInfo()
        self._check(self.L.icr_get_factor_info(self._h, C.byref(info)))
        return {k: getattr(info, k) for k, _ in FactorInfo._fields_}

    def set_candidates(self, nodes, mu):
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        self._check(self.L.icr_set_candidates(self._h, len(nodes), _np_ptr(nodes), _np_ptr(mu)))

    def set_pairs(self, ids, weights, normals, mu):
        ids = np.ascontiguousarray(ids, dtype=np.int32).reshape(-1, 4)
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1, 4)
        nrm = np.ascontiguousarray(normals, dtype=np.float64).reshape(-1, 3)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        self._check(self.L.icr_set_pairs(self._h, len(ids), _np_ptr(ids), _np_ptr(w), _np_ptr(nrm), _np_ptr(mu)))

    # -- hot-path calls ------------------------------------------------------
    def build_WH(self, node_ids, WH, weights=None):
        """Nodal contacts (node_ids [n_c]) or, with weights, mapped contacts
        (node_ids and weights [n_c, 4], -1 = unused slot)."""
        t = self._torch
        if weights is None:
            nc = node_ids.numel()
            wp = None
        else:
            nc = node_ids.numel() // 4
            if weights.numel() != 4 * nc or node_ids.numel() != 4 * nc:
                raise ValueError("mapped contacts need node_ids and weights of 4 entries per contact")
            wp = _dptr(weights, t.float64)
        self._check(self.L.icr_build_WH(self._h, nc, _dptr(node_ids, t.int32), wp,
                                        _dptr(WH, t.float64, 9 * nc * nc)))

    def update_W(self, WH, Cm, W):
        t = self._torch
        nc = Cm.numel() // 9
        self._check(self.L.icr_update_W(self._h, nc, _dptr(WH, t.float64, 9 * nc * nc), _dptr(Cm, t.float64),
                                        _dptr(W, t.float64, 9 * nc * nc)))

    def solve_contacts(self, W, d, mu, h, lam, status, max_sweeps, tol, j_inner=8, sync=True):
        t = self._torch
        nc = mu.numel()
        sw, ep = C.c_int32(0), C.c_double(0.0)
        st = self.L.icr_solve_contacts(self._h, nc, _dptr(W, t.float64, 9 * nc * nc), _dptr(d, t.float64, 3 * nc),
                                       _dptr(mu, t.float64), h, _dptr(lam, t.float64, 3 * nc),
                                       _dptr(status, t.int8, nc), max_sweeps, tol, j_inner,
                                       C.byref(sw) if sync else None, C.byref(ep) if sync else None)
        self._check(st, allow_warn=True)
        return (sw.value, ep.value) if sync else (None, None)

    def proximity_update(self, WH, p_free, f, h, p):
        t = self._torch
        nc = p_free.numel() // 3
        self._check(self.L.icr_proximity_update(self._h, nc, _dptr(WH, t.float64, 9 * nc * nc),
                                                _dptr(p_free, t.float64), _dptr(f, t.float64), h,
                                                _dptr(p, t.float64)))

    def step(self, obstacle, n_contacts, n_newton=5, max_sweeps=200, tol=1e-10, j_inner=8, timing=False,
             report=True, standard=False, graph=True, per_constraint=False, precision=FP64, refine=1):
        ob = _obstacle(obstacle)
        scheme = 1 if standard else (2 if per_constraint else 0)
        op = StepOpts(n_contacts, n_newton, max_sweeps, j_inner, tol, 1 if timing else 0, scheme,
                      1 if graph else 0, int(precision), int(refine))
        rep = StepReport()
        self._check(self.L.icr_step(self._h, C.byref(ob), C.byref(op), C.byref(rep) if report else None))
        if not report:
            return None
        out = {k: getattr(rep, k) for k, _ in StepReport._fields_}
        out["sweeps"] = list(rep.sweeps)[:n_newton]
        out["eps"] = list(rep.eps)[:n_newton]
        return out

    def reserve(self, max_contacts, precision=FP64):
        self._check(self.L.icr_reserve(self._h, int(max_contacts), int(precision)))

    def get_state(self):
        t = self._torch
        q = t.empty(self.n, dtype=t.float64, device="cuda")
        v = t.empty(self.n, dtype=t.float64, device="cuda")
        tt = C.c_double(0.0)
        self._check(self.L.icr_get_state(self._h, _dptr(q), _dptr(v), C.byref(tt)))
        return q, v, tt.value

    def set_state(self, q, v, time):
        self._check(self.L.icr_set_state(self._h, _dptr(q, self._torch.float64, self.n),
                                         _dptr(v, self._torch.float64, self.n), time))

    def step_results(self, nc, with_WH=False):
        t = self._torch
        dev = "cuda"
        m = 3 * nc
        out = dict(node_ids=t.empty(nc, dtype=t.int32, device=dev), q_free=t.empty(self.n, dtype=t.float64, device=dev),
                   p=t.empty(m, dtype=t.float64, device=dev), lam=t.empty(m, dtype=t.float64, device=dev),
                   C=t.empty(9 * nc, dtype=t.float64, device=dev), f=t.empty(m, dtype=t.float64, device=dev),
                   status=t.empty(nc, dtype=t.int8, device=dev))
        WH = t.empty(m * m, dtype=t.float64, device=dev) if with_WH else None
        self._check(self.L.icr_get_step_results(self._h, _dptr(out["node_ids"]), _dptr(out["q_free"]),
                                                _dptr(out["p"]), _dptr(out["lam"]), _dptr(out["C"]),
                                                _dptr(out["f"]), _dptr(out["status"]),
                                                _dptr(WH) if with_WH else None))
        if with_WH:
            out["WH"] = WH
        return out


def _obstacle(obstacle):
    ob = Obstacle()
    ob.kind = 1 if obstacle["kind"] == "sphere" else 0
    for i in range(3):
        ob.c0[i] = float(obstacle["c0"][i])
        ob.vel[i] = float(obstacle["vel"][i])
        ob.normal[i] = float(obstacle["normal"][i])
    ob.radius = float(obstacle.get("radius", 0.0))
    return ob


class Server:
    """Serving runtime over many admitted scenes (wraps an icr_server handle)."""

    def __init__(self, hbm_budget, slots=4, batching=8, max_wait_ms=0.0):
        """batching: requests per slot and round with batched Newton loops
        (True = 8), or 0 / False for one whole icr_step per slot; a short
        group waits up to max_wait_ms for more requests while a slot runs."""
        self.L = lib()
        h = C.c_void_p()
        st = self.L.icr_server_create(C.byref(h), int(hbm_budget), int(slots))
        if st != OK:
            raise IcrError(st, "icr_server_create failed")
        self._h = h
        self._scenes = {}
        group = 8 if batching is True else int(batching)
        self._check(self.L.icr_server_set_batching(self._h, group, float(max_wait_ms)))

    def _check(self, st):
        if st != OK:
            raise IcrError(st, self.L.icr_server_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.L.icr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, scene):
        sid = C.c_int32(0)
        self._check(self.L.icr_server_admit(self._h, scene._h, C.byref(sid)))
        self._scenes[sid.value] = scene
        return sid.value

    def evict(self, sid):
        self._check(self.L.icr_server_evict(self._h, int(sid)))
        self._scenes.pop(sid, None)

    def used(self):
        b = C.c_int64(0)
        self._check(self.L.icr_server_used(self._h, C.byref(b)))
        return b.value

    def submit(self, sid, obstacle, n_contacts, n_newton=5, max_sweeps=200, tol=1e-10, j_inner=8, tag=0,
               graph=True, precision=FP64, refine=1):
        op = StepOpts(n_contacts, n_newton, max_sweeps, j_inner, tol, 0, 0, 1 if graph else 0, int(precision),
                      int(refine))
        self._check(self.L.icr_server_submit(self._h, int(sid), C.byref(_obstacle(obstacle)), C.byref(op),
                                             C.c_uint64(tag)))

    def poll(self, wait=False, cap=256):
        """Launch what fits, return (completions, pending) with completions as dicts."""
        out = (Completion * cap)()
        n, pend = C.c_int32(0), C.c_int32(0)
        self._check(self.L.icr_server_poll(self._h, out, cap, C.byref(n), 1 if wait else 0, C.byref(pend)))
        res = [dict(tag=out[i].tag, scene=out[i].scene, status=out[i].status, latency_ms=out[i].latency_ms,
                    queue_ms=out[i].queue_ms) for i in range(n.value)]
        return res, pend.value


def scene_from_dict(sc, stream=None):
    """Create, assemble, factor and set candidates for a generator scene."""
    s = Scene(stream)
    s.assemble(sc)
    s.factor()
    if sc.get("pairs") is not None:
        pr = sc["pairs"]
        s.set_pairs(pr["ids"], pr["w"], pr["normals"], pr["mu"])
    s.set_candidates(sc["candidates"], sc["cand_mu"])
    return s
