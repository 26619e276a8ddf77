"""ctypes binding of librp.so: argument marshalling only.

Every function here has the name of the C entry point it calls and forwards
its arguments: torch tensors become device pointers, numpy arrays become
host pointers.  All arithmetic runs in the library's HIP kernels; there is no
CPU fallback, and a missing library raises on import.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .build import library_path

RP_OK = 0
RP_FP64 = 0
RP_SPLIT_BF16 = 1
RP_SPLIT_BF16_X6 = 2
RP_W_TETRA = 0
RP_W_SAMPLING = 1
RP_W_TETRA_METAL = 2

STATUS_NAMES = {0: "RP_OK", 1: "RP_E_NULL", 2: "RP_E_SHAPE", 3: "RP_E_RANGE", 4: "RP_E_ALIAS",
                5: "RP_E_NOMEM", 6: "RP_E_DEVICE", 7: "RP_E_SINGULAR", 8: "RP_E_UNSUPPORTED"}

EXPORTED = ["rp_create", "rp_destroy", "rp_synchronize", "rp_last_error", "rp_pair_density",
            "rp_weights", "rp_chi0_accumulate", "rp_chi0_accumulate_noalloc", "rp_chi0_batch", "rp_chi0_batch_graphs", "rp_chi0_run", "rp_screen_W", "rp_wannier_W",
            "rp_set_tuning", "rp_head_density", "rp_screen_head", "rp_wannier_qterm",
            "rp_coulomb_cell_average", "rp_frequency_grid", "rp_unfold_coef", "rp_unfold_eps_inv",
            "rp_set_fermi_level", "rp_pair_grid", "rp_plasma_frequency", "rp_set_drude", "rp_profile",
            "rp_profile_read"]

STAGES = ["ugrid", "pair", "weights", "prep", "chi", "screen", "wannier", "batch", "unfold", "reduce"]


class RpError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class rp_cell(ctypes.Structure):
    _fields_ = [("lat", (ctypes.c_double * 3) * 3), ("fft", ctypes.c_int * 3),
                ("kmesh", ctypes.c_int * 3)]


class rp_problem(ctypes.Structure):
    """One chi0 problem of rp_chi0_batch (the C struct of the same name)."""
    _fields_ = [("cell", rp_cell), ("iq", ctypes.c_int * 3), ("nband", ctypes.c_int),
                ("npw_max", ctypes.c_int), ("npw", ctypes.c_void_p), ("mmax", ctypes.c_int * 3),
                ("miller", ctypes.c_void_p), ("coef", ctypes.c_void_p), ("energy_eV", ctypes.c_void_p),
                ("T", ctypes.c_void_p), ("o0", ctypes.c_int), ("o1", ctypes.c_int), ("e0", ctypes.c_int),
                ("e1", ctypes.c_int), ("k0", ctypes.c_int), ("k1", ctypes.c_int), ("ng", ctypes.c_int),
                ("gsph", ctypes.c_void_p), ("nfreq", ctypes.c_int), ("freq_eV", ctypes.c_void_p),
                ("delta_eV", ctypes.c_double), ("wm", ctypes.c_int), ("kbatch", ctypes.c_int),
                ("accumulate", ctypes.c_int), ("chi", ctypes.c_void_p)]


class rp_tune_entry(ctypes.Structure):
    """One size class of the launch-shape table (the C struct of the same name)."""
    _fields_ = [("ng_max", ctypes.c_int), ("grid_max", ctypes.c_int), ("chi_nw", ctypes.c_int),
                ("chi_fill", ctypes.c_int), ("fft_lines", ctypes.c_int), ("chi_kernel", ctypes.c_int)]


TUNE_FIELDS = [f[0] for f in rp_tune_entry._fields_]


def make_cell(lat, fft, kmesh) -> rp_cell:
    c = rp_cell()
    lat = np.asarray(lat, dtype=np.float64)
    for i in range(3):
        for j in range(3):
            c.lat[i][j] = float(lat[i, j])
        c.fft[i] = int(fft[i])
        c.kmesh[i] = int(kmesh[i])
    return c


_LIB = None


def load(path: Optional[str] = None):
    """Load librp.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2001_02351_amd/build.py "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    cellp = ctypes.POINTER(rp_cell)
    sig = {
        "rp_create": [ctypes.POINTER(P), I, P],
        "rp_destroy": [P],
        "rp_synchronize": [P],
        "rp_pair_density": [P, cellp, P, I, I, P, P, P, P, I, I, I, I, I, I, I, P, I, P],
        "rp_weights": [P, cellp, P, I, P, P, I, I, I, I, I, I, I, P, D, I, P],
        "rp_chi0_accumulate": [P, cellp, P, I, P, P, I, I, I, I, I, I, I, P, I, P, D, I, I, I, P],
        "rp_chi0_accumulate_noalloc": [P, cellp, P, I, P, P, I, I, I, I, I, I, I, P, I, P, D, I, I, I, P],
        "rp_chi0_batch": [P, I, ctypes.POINTER(rp_problem), I],
        "rp_chi0_batch_graphs": [P, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_long)],
        "rp_chi0_run": [P, ctypes.POINTER(rp_problem), I],
        "rp_screen_W": [P, cellp, P, I, P, I, P, P, P],
        "rp_wannier_W": [P, cellp, P, I, P, P, I, P, I, P, I, P, P],
        "rp_set_tuning": [P, I, ctypes.POINTER(rp_tune_entry)],
        "rp_head_density": [P, cellp, I, I, P, P, P, P, I, I, I, I, I, I, P, I, I, P],
        "rp_screen_head": [P, cellp, I, P, I, P, P, P, P],
        "rp_wannier_qterm": [P, cellp, P, I, P, P, I, P, I, P, I, P, I, P, I, P, P, P, P],
        "rp_coulomb_cell_average": [cellp, ctypes.POINTER(D)],
        "rp_frequency_grid": [D, D, I, I, P],
        "rp_unfold_coef": [P, cellp, P, P, P, I, I, P, P, ctypes.c_long, P, I, P, P, ctypes.c_long],
        "rp_unfold_eps_inv": [P, cellp, P, P, P, I, P, P, I, P, I, P, P],
        "rp_set_fermi_level": [P, D],
        "rp_pair_grid": [cellp, P, P, I, P, I, P],
        "rp_plasma_frequency": [P, cellp, I, I, P, P, P, P, P, I, I, D, P],
        "rp_set_drude": [P, D, D],
        "rp_profile": [P, I],
        "rp_profile_read": [P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.rp_last_error.argtypes = [P]
    lib.rp_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _hp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dp(t) -> Optional[int]:
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _need(t, name: str, kind: str, n: int, optional: bool = False):
    """Checks that device tensor t holds at least n elements of kind "f64"
    (float64; complex arrays as interleaved pairs) or "i32", so the library
    never reads or writes past its end."""
    import torch
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    want = torch.float64 if kind == "f64" else torch.int32
    if t.dtype != want:
        raise ValueError(f"{name}: expected {want}, got {t.dtype}")
    if t.numel() < n:
        raise ValueError(f"{name}: {t.numel()} elements, the call needs {n}")


def _nk(cell) -> int:
    return int(cell.kmesh[0]) * int(cell.kmesh[1]) * int(cell.kmesh[2])


def _nr(cell) -> int:
    return int(cell.fft[0]) * int(cell.fft[1]) * int(cell.fft[2])


def _pairs(o0, o1, e0, e1, k0, k1) -> int:
    return max(0, k1 - k0) * max(0, e1 - e0) * max(0, o1 - o0)


def _bands(cell, nband, npw_max, miller, coef):
    _need(miller, "miller", "i32", _nk(cell) * int(npw_max) * 3)
    _need(coef, "coef", "f64", _nk(cell) * int(nband) * int(npw_max) * 2)


DEFAULT_TUNING = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json")


def load_tuning(path: str) -> list:
    """The entries of a tuning table written by the autotuner."""
    import json
    with open(path) as f:
        table = json.load(f)
    entries = table["entries"]
    for e in entries:
        if sorted(e) != sorted(TUNE_FIELDS):
            raise ValueError(f"{path}: entry fields {sorted(e)} != {sorted(TUNE_FIELDS)}")
    return entries


class Context:
    """An rp_ctx bound to a dedicated default-priority torch stream.

    tuning: "default" installs the package's measured table when it exists,
    a path installs that table, None leaves the library's defaults."""

    def __init__(self, device: int = 0, tuning: Optional[str] = "default"):
        import torch
        self.lib = load()
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        h = ctypes.c_void_p()
        st = self.lib.rp_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if st != RP_OK:
            raise RpError(st, "rp_create", "context creation failed")
        self.handle = h
        self.tuning = None
        path = DEFAULT_TUNING if tuning == "default" else tuning
        if path is not None and (tuning != "default" or os.path.exists(path)):
            rp_set_tuning(self, load_tuning(path))
            self.tuning = path

    def close(self):
        if getattr(self, "handle", None):
            self.lib.rp_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, where: str):
        if st != RP_OK:
            raise RpError(st, where, self.lib.rp_last_error(self.handle).decode())

    def _enter(self):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        import torch
        torch.cuda.current_stream(self.device).wait_stream(self.stream)


def rp_synchronize(ctx: Context):
    ctx._check(ctx.lib.rp_synchronize(ctx.handle), "rp_synchronize")


def rp_last_error(ctx: Context) -> str:
    return ctx.lib.rp_last_error(ctx.handle).decode()


def rp_pair_density(ctx: Context, cell: rp_cell, iq, nband, npw_max, npw, mmax, miller, coef,
                    o0, o1, e0, e1, k0, k1, ng, gsph, prec, M):
    iq_h, npw_h, mm_h = _host(iq, np.int32), _host(npw, np.int32), _host(mmax, np.int32)
    g_h = _host(gsph, np.int32)
    _bands(cell, nband, npw_max, miller, coef)
    _need(M, "M", "f64", _pairs(o0, o1, e0, e1, k0, k1) * int(ng) * 2)
    ctx._enter()
    st = ctx.lib.rp_pair_density(ctx.handle, ctypes.byref(cell), _hp(iq_h), int(nband), int(npw_max),
                                 _hp(npw_h), _hp(mm_h), _dp(miller), _dp(coef), o0, o1, e0, e1, k0, k1,
                                 int(ng), _hp(g_h), int(prec), _dp(M))
    ctx._leave()
    ctx._check(st, "rp_pair_density")


def rp_weights(ctx: Context, cell: rp_cell, iq, nband, energy_eV, T, o0, o1, e0, e1, k0, k1, nfreq,
               freq_eV, delta_eV, wm, w):
    iq_h, f_h = _host(iq, np.int32), _host(freq_eV, np.complex128)
    _need(energy_eV, "energy_eV", "f64", _nk(cell) * int(nband))
    _need(T, "T", "f64", _nk(cell) * int(nband), optional=True)
    _need(w, "w", "f64", int(nfreq) * _pairs(o0, o1, e0, e1, k0, k1) * 2)
    ctx._enter()
    st = ctx.lib.rp_weights(ctx.handle, ctypes.byref(cell), _hp(iq_h), int(nband), _dp(energy_eV),
                            _dp(T), o0, o1, e0, e1, k0, k1, int(nfreq), _hp(f_h), float(delta_eV),
                            int(wm), _dp(w))
    ctx._leave()
    ctx._check(st, "rp_weights")


def _chi_args(cell, nband, energy_eV, T, o0, o1, e0, e1, k0, k1, ng, M, nfreq, chi):
    _need(energy_eV, "energy_eV", "f64", _nk(cell) * int(nband))
    _need(T, "T", "f64", _nk(cell) * int(nband), optional=True)
    _need(M, "M", "f64", _pairs(o0, o1, e0, e1, k0, k1) * int(ng) * 2)
    _need(chi, "chi", "f64", int(nfreq) * int(ng) * int(ng) * 2)


def rp_chi0_accumulate(ctx: Context, cell: rp_cell, iq, nband, energy_eV, T, o0, o1, e0, e1, k0, k1,
                       ng, M, nfreq, freq_eV, delta_eV, wm, prec, accumulate, chi):
    iq_h, f_h = _host(iq, np.int32), _host(freq_eV, np.complex128)
    _chi_args(cell, nband, energy_eV, T, o0, o1, e0, e1, k0, k1, ng, M, nfreq, chi)
    ctx._enter()
    st = ctx.lib.rp_chi0_accumulate(ctx.handle, ctypes.byref(cell), _hp(iq_h), int(nband),
                                    _dp(energy_eV), _dp(T), o0, o1, e0, e1, k0, k1, int(ng), _dp(M),
                                    int(nfreq), _hp(f_h), float(delta_eV), int(wm), int(prec),
                                    int(accumulate), _dp(chi))
    ctx._leave()
    ctx._check(st, "rp_chi0_accumulate")


def rp_chi0_accumulate_noalloc(ctx: Context, cell: rp_cell, iq, nband, energy_eV, T, o0, o1, e0, e1, k0, k1,
                               ng, M, nfreq, freq_eV, delta_eV, wm, prec, accumulate, chi):
    iq_h, f_h = _host(iq, np.int32), _host(freq_eV, np.complex128)
    _chi_args(cell, nband, energy_eV, T, o0, o1, e0, e1, k0, k1, ng, M, nfreq, chi)
    ctx._enter()
    st = ctx.lib.rp_chi0_accumulate_noalloc(ctx.handle, ctypes.byref(cell), _hp(iq_h), int(nband),
                                            _dp(energy_eV), _dp(T), o0, o1, e0, e1, k0, k1, int(ng), _dp(M),
                                            int(nfreq), _hp(f_h), float(delta_eV), int(wm), int(prec),
                                            int(accumulate), _dp(chi))
    ctx._leave()
    ctx._check(st, "rp_chi0_accumulate_noalloc")


def _fill_problem(r, q, keep):
    """Fills the rp_problem r from the dict q (host copies appended to keep)."""
    r.cell = q["cell"]
    for a in range(3):
        r.iq[a] = int(q["iq"][a])
    npw_h, mm_h = _host(q["npw"], np.int32), _host(q["mmax"], np.int32)
    g_h, f_h = _host(q["gsph"], np.int32), _host(q["freq_eV"], np.complex128)
    keep += [npw_h, g_h, f_h]
    for a in range(3):
        r.mmax[a] = int(mm_h[a])
    r.npw, r.gsph, r.freq_eV = _hp(npw_h), _hp(g_h), _hp(f_h)
    _bands(q["cell"], q["nband"], q["npw_max"], q["miller"], q["coef"])
    _need(q["energy_eV"], "energy_eV", "f64", _nk(q["cell"]) * int(q["nband"]))
    _need(q.get("T"), "T", "f64", _nk(q["cell"]) * int(q["nband"]), optional=True)
    _need(q["chi"], "chi", "f64", int(q["nfreq"]) * int(q["ng"]) ** 2 * 2)
    r.miller, r.coef = _dp(q["miller"]), _dp(q["coef"])
    r.energy_eV, r.T, r.chi = _dp(q["energy_eV"]), _dp(q.get("T")), _dp(q["chi"])
    for name in ("nband", "npw_max", "o0", "o1", "e0", "e1", "k0", "k1", "ng", "nfreq", "wm",
                 "kbatch", "accumulate"):
        setattr(r, name, int(q[name]))
    r.delta_eV = float(q["delta_eV"])


def rp_chi0_batch(ctx: Context, problems, prec):
    """problems: a sequence of dicts with the rp_problem fields; "cell" is an
    rp_cell, host arrays (npw, mmax, gsph, freq_eV) are numpy-convertible,
    device arrays (miller, coef, energy_eV, T, chi) are torch tensors."""
    keep = []
    arr = (rp_problem * max(1, len(problems)))()
    for i, q in enumerate(problems):
        _fill_problem(arr[i], q, keep)
    ctx._enter()
    st = ctx.lib.rp_chi0_batch(ctx.handle, len(problems), arr, int(prec))
    ctx._leave()
    ctx._check(st, "rp_chi0_batch")


def rp_chi0_run(ctx: Context, problem, prec):
    """One problem (a dict as for rp_chi0_batch), enqueued without a graph."""
    keep = []
    r = rp_problem()
    _fill_problem(r, problem, keep)
    ctx._enter()
    st = ctx.lib.rp_chi0_run(ctx.handle, ctypes.byref(r), int(prec))
    ctx._leave()
    ctx._check(st, "rp_chi0_run")


def rp_chi0_batch_graphs(ctx: Context) -> tuple:
    """(graphs, kernel nodes) of the most recent rp_chi0_batch capture."""
    g, n = ctypes.c_int(0), ctypes.c_long(0)
    ctx._check(ctx.lib.rp_chi0_batch_graphs(ctx.handle, ctypes.byref(g), ctypes.byref(n)), "rp_chi0_batch_graphs")
    return g.value, n.value


def rp_head_density(ctx: Context, cell: rp_cell, nband, npw_max, npw, miller, coef, energy_eV, o0, o1, e0, e1,
                    k0, k1, qhat, ng, col, M):
    npw_h, q_h = _host(npw, np.int32), _host(qhat, np.float64)
    _bands(cell, nband, npw_max, miller, coef)
    _need(energy_eV, "energy_eV", "f64", _nk(cell) * int(nband))
    _need(M, "M", "f64", _pairs(o0, o1, e0, e1, k0, k1) * int(ng) * 2)
    ctx._enter()
    st = ctx.lib.rp_head_density(ctx.handle, ctypes.byref(cell), int(nband), int(npw_max), _hp(npw_h), _dp(miller),
                                 _dp(coef), _dp(energy_eV), o0, o1, e0, e1, k0, k1, _hp(q_h), int(ng), int(col),
                                 _dp(M))
    ctx._leave()
    ctx._check(st, "rp_head_density")


def rp_screen_head(ctx: Context, cell: rp_cell, ng, gsph, nfreq, freq_eV, chi, eps_inv, optics):
    g_h, f_h = _host(gsph, np.int32), _host(freq_eV, np.complex128)
    n2 = int(nfreq) * int(ng) * int(ng) * 2
    _need(chi, "chi", "f64", n2)
    _need(eps_inv, "eps_inv", "f64", n2, optional=True)
    _need(optics, "optics", "f64", int(nfreq) * 5, optional=True)
    ctx._enter()
    st = ctx.lib.rp_screen_head(ctx.handle, ctypes.byref(cell), int(ng), _hp(g_h), int(nfreq), _hp(f_h), _dp(chi),
                                _dp(eps_inv), _dp(optics))
    ctx._leave()
    ctx._check(st, "rp_screen_head")


def rp_screen_W(ctx: Context, cell: rp_cell, iq, ng, gsph, nfreq, chi, eps_inv, W):
    iq_h, g_h = _host(iq, np.int32), _host(gsph, np.int32)
    n2 = int(nfreq) * int(ng) * int(ng) * 2
    _need(chi, "chi", "f64", n2)
    _need(eps_inv, "eps_inv", "f64", n2, optional=True)
    _need(W, "W", "f64", n2, optional=True)
    ctx._enter()
    st = ctx.lib.rp_screen_W(ctx.handle, ctypes.byref(cell), _hp(iq_h), int(ng), _hp(g_h), int(nfreq),
                             _dp(chi), _dp(eps_inv), _dp(W))
    ctx._leave()
    ctx._check(st, "rp_screen_W")


def rp_wannier_W(ctx: Context, cell: rp_cell, iq, nwan, phi, centre_frac, ng, gsph, ntail, gtail,
                 nfreq, eps_inv, Wij):
    iq_h, c_h = _host(iq, np.int32), _host(centre_frac, np.float64)
    g_h = _host(gsph, np.int32)
    t_h = _host(gtail, np.int32) if ntail > 0 else None
    _need(phi, "phi", "f64", int(nwan) * _nr(cell))
    _need(eps_inv, "eps_inv", "f64", int(nfreq) * int(ng) * int(ng) * 2)
    _need(Wij, "Wij", "f64", int(nfreq) * int(nwan) * int(nwan) * 2)
    ctx._enter()
    st = ctx.lib.rp_wannier_W(ctx.handle, ctypes.byref(cell), _hp(iq_h), int(nwan), _dp(phi), _hp(c_h),
                              int(ng), _hp(g_h), int(ntail), _hp(t_h), int(nfreq), _dp(eps_inv), _dp(Wij))
    ctx._leave()
    ctx._check(st, "rp_wannier_W")


def rp_wannier_qterm(ctx: Context, cell: rp_cell, iq, nwan, phi, centre_frac, R, ng, gsph, ntail, gtail,
                     nfreq, eps_inv, accumulate, U=None, J=None, V=None, X=None):
    """One q-point's term of the q-sums of U, J (c128 [nfreq][nR][nwan][nwan]) and
    V, X (c128 [nR][nwan][nwan]); any output may be None."""
    iq_h, c_h = _host(iq, np.int32), _host(centre_frac, np.float64)
    R_h = _host(R, np.int32).reshape(-1, 3)
    g_h = _host(gsph, np.int32)
    t_h = _host(gtail, np.int32) if ntail > 0 else None
    nR = int(R_h.shape[0])
    _need(phi, "phi", "f64", int(nwan) * _nr(cell))
    _need(eps_inv, "eps_inv", "f64", int(nfreq) * int(ng) * int(ng) * 2)
    for name, t, n in (("U", U, int(nfreq) * nR), ("J", J, int(nfreq) * nR), ("V", V, nR), ("X", X, nR)):
        _need(t, name, "f64", n * int(nwan) * int(nwan) * 2, optional=True)
    ctx._enter()
    st = ctx.lib.rp_wannier_qterm(ctx.handle, ctypes.byref(cell), _hp(iq_h), int(nwan), _dp(phi), _hp(c_h),
                                  int(R_h.shape[0]), _hp(R_h), int(ng), _hp(g_h), int(ntail), _hp(t_h),
                                  int(nfreq), _dp(eps_inv), int(accumulate), _dp(U), _dp(J), _dp(V), _dp(X))
    ctx._leave()
    ctx._check(st, "rp_wannier_qterm")


def rp_coulomb_cell_average(cell: rp_cell) -> float:
    """Mean of 1/|q|^2 over the q-cell around Gamma (host computation; no
    context or device needed)."""
    out = ctypes.c_double(0.0)
    st = load().rp_coulomb_cell_average(ctypes.byref(cell), ctypes.byref(out))
    if st != 0:
        raise RpError(st, "rp_coulomb_cell_average", "invalid cell")
    return out.value


def rp_plasma_frequency(ctx, cell: rp_cell, nband: int, npw_max: int, npw, miller, coef, energy_eV, T, b0: int,
                        b1: int, ef_eV: float) -> np.ndarray:
    """The intraband plasma tensor Omega^{mu nu} (eV^2, 3 x 3) of bands [b0, b1)."""
    npw_h = _host(npw, np.int32)
    out = np.zeros(9, np.float64)
    _bands(cell, nband, npw_max, miller, coef)
    _need(energy_eV, "energy_eV", "f64", _nk(cell) * int(nband))
    _need(T, "T", "f64", _nk(cell) * int(nband), optional=True)
    ctx._enter()
    st = ctx.lib.rp_plasma_frequency(ctx.handle, ctypes.byref(cell), int(nband), int(npw_max), _hp(npw_h),
                                     _dp(miller), _dp(coef), _dp(energy_eV), _dp(T), int(b0), int(b1), float(ef_eV),
                                     _hp(out))
    ctx._leave()
    ctx._check(st, "rp_plasma_frequency")
    return out.reshape(3, 3)


def rp_set_drude(ctx, wq_eV2: float, delta_eV: float) -> None:
    """The intraband head term wq = qhat.Omega.qhat (eV^2) and its broadening
    for rp_screen_head; wq = 0 removes it."""
    ctx._check(ctx.lib.rp_set_drude(ctx.handle, float(wq_eV2), float(delta_eV)), "rp_set_drude")


def rp_pair_grid(cell: rp_cell, iq, mmax, gsph, prec: int) -> tuple:
    """The grid (N1, N2, N3) that the pair densities are built on for these
    arguments (host computation; no context or device needed)."""
    iq_h, mm_h, g_h = _host(iq, np.int32), _host(mmax, np.int32), _host(gsph, np.int32)
    out = np.zeros(3, np.int32)
    st = load().rp_pair_grid(ctypes.byref(cell), _hp(iq_h), _hp(mm_h), int(g_h.shape[0]), _hp(g_h), int(prec),
                             _hp(out))
    if st != 0:
        raise RpError(st, "rp_pair_grid", STATUS_NAMES.get(st, str(st)))
    return tuple(int(x) for x in out)


def rp_frequency_grid(emax_eV: float, dw_eV: float = 0.05, nomega: int = 70, nmax: int = 0) -> np.ndarray:
    """The logarithmic frequency grid (eV), host computation; nmax = 0 takes
    9 nomega / 10."""
    out = np.zeros(max(0, int(nomega)), np.float64)
    st = load().rp_frequency_grid(float(emax_eV), float(dw_eV), int(nomega), int(nmax), _hp(out) if out.size else None)
    if st != 0:
        raise RpError(st, "rp_frequency_grid", "invalid grid parameters")
    return out


def _op(W, t):
    return _host(W, np.int32).reshape(9), _host(t, np.float64).reshape(3)


def _ld(t) -> int:
    """Leading dimension (complex elements) of a [n][ld][2] or [n][2 ld] tensor."""
    return int(t.shape[1]) if t.dim() == 3 else int(t.shape[1]) // 2


def rp_unfold_coef(ctx: Context, cell: rp_cell, W, t, ik_irr, miller_irr, coef_irr, ik, miller, coef):
    """coef_irr and coef: device tensors [nband][ld][2] or [nband][2 ld]
    (interleaved complex); miller lists host int [n][3]."""
    W_h, t_h = _op(W, t)
    mi, mt = _host(miller_irr, np.int32).reshape(-1, 3), _host(miller, np.int32).reshape(-1, 3)
    ki, kt = _host(ik_irr, np.int32), _host(ik, np.int32)
    _need(coef_irr, "coef_irr", "f64", int(coef_irr.shape[0]) * _ld(coef_irr) * 2)
    _need(coef, "coef", "f64", int(coef_irr.shape[0]) * _ld(coef) * 2)
    ctx._enter()
    st = ctx.lib.rp_unfold_coef(ctx.handle, ctypes.byref(cell), _hp(W_h), _hp(t_h), _hp(ki), int(coef_irr.shape[0]),
                                int(mi.shape[0]), _hp(mi), _dp(coef_irr), _ld(coef_irr), _hp(kt),
                                int(mt.shape[0]), _hp(mt), _dp(coef), _ld(coef))
    ctx._leave()
    ctx._check(st, "rp_unfold_coef")


def rp_unfold_eps_inv(ctx: Context, cell: rp_cell, W, t, iq_irr, gsph_irr, iq, gsph, src, dst):
    """src [nfreq][ng_irr][ng_irr][2], dst [nfreq][ng][ng][2] device tensors."""
    W_h, t_h = _op(W, t)
    gi, gt = _host(gsph_irr, np.int32).reshape(-1, 3), _host(gsph, np.int32).reshape(-1, 3)
    qi, qt = _host(iq_irr, np.int32), _host(iq, np.int32)
    nf = int(src.shape[0])
    _need(src, "src", "f64", nf * int(gi.shape[0]) ** 2 * 2)
    _need(dst, "dst", "f64", nf * int(gt.shape[0]) ** 2 * 2)
    ctx._enter()
    st = ctx.lib.rp_unfold_eps_inv(ctx.handle, ctypes.byref(cell), _hp(W_h), _hp(t_h), _hp(qi), int(gi.shape[0]),
                                   _hp(gi), _hp(qt), int(gt.shape[0]), _hp(gt), int(src.shape[0]), _dp(src), _dp(dst))
    ctx._leave()
    ctx._check(st, "rp_unfold_eps_inv")


def rp_set_fermi_level(ctx: Context, ef_eV: float):
    """Fermi level (eV) of the RP_W_TETRA_METAL weights; nan clears it."""
    ctx._check(ctx.lib.rp_set_fermi_level(ctx.handle, float(ef_eV)), "rp_set_fermi_level")


def rp_set_tuning(ctx: Context, entries):
    """entries: a sequence of dicts with the rp_tune_entry fields (empty clears)."""
    arr = (rp_tune_entry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        for name in TUNE_FIELDS:
            setattr(arr[i], name, int(e[name]))
    ctx._check(ctx.lib.rp_set_tuning(ctx.handle, len(entries), arr), "rp_set_tuning")


def rp_profile(ctx: Context, enable: bool):
    ctx._check(ctx.lib.rp_profile(ctx.handle, int(bool(enable))), "rp_profile")


def rp_profile_read(ctx: Context) -> dict:
    """{stage: (milliseconds, launches)} accumulated since rp_profile(ctx, True)."""
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_long * len(STAGES))()
    ctx._check(ctx.lib.rp_profile_read(ctx.handle, ms, cnt), "rp_profile_read")
    return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}
