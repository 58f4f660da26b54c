"""ctypes binding of libfrbx.so (C ABI declared in include/frbx.h).

Argument marshalling only: every step of the search runs inside the
library.  PyTorch supplies device memory and the HIP stream.  The library
must have been built (``python -m paper_1801_02391_amd.build``); loading
raises if it is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfrbx.so")
_lib = None

OK, E_INVAL, E_STATE, E_RANGE, E_NOMEM, E_DEVICE = range(6)
PREC_F32, PREC_F16X3, PREC_F16 = 0, 1, 2
PRECISIONS = {"f32": PREC_F32, "f16x3": PREC_F16X3, "f16": PREC_F16}
_STATUS = {0: "OK", 1: "E_INVAL", 2: "E_STATE", 3: "E_RANGE", 4: "E_NOMEM", 5: "E_DEVICE"}


class FrbxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Layout(C.Structure):
    _fields_ = [("n_baselines", C.c_int32), ("n_if", C.c_int32), ("n_chan", C.c_int32),
                ("n_frames", C.c_int64), ("t_ap_ms", C.c_double), ("chan_bw_mhz", C.c_double),
                ("if_freq_mhz", C.POINTER(C.c_double))]


class Candidate(C.Structure):
    _fields_ = [("baseline", C.c_int32), ("dm_index", C.c_int32), ("window_index", C.c_int32),
                ("window_len", C.c_int32), ("segment", C.c_int64), ("k0", C.c_int64),
                ("dm", C.c_double), ("power", C.c_double), ("power_norm", C.c_double),
                ("rate_idx", C.c_int32), ("sbd_idx", C.c_int32), ("mbd_idx", C.c_int32),
                ("n_windows", C.c_int32), ("rate", C.c_double), ("sbd_us", C.c_double),
                ("mbd_us", C.c_double), ("group_id", C.c_int32), ("reserved", C.c_int32)]


class Group(C.Structure):
    _fields_ = [("group_id", C.c_int32), ("n_baselines", C.c_int32), ("k_start", C.c_int64),
                ("k_end", C.c_int64), ("best", C.c_int32), ("reported", C.c_int32)]


class Timing(C.Structure):
    _fields_ = [("fringe_ms", C.c_double), ("n_fringe", C.c_int64), ("fringe_units", C.c_int64),
                ("dedisperse_ms", C.c_double), ("n_dedisperse", C.c_int64),
                ("dedisperse_units", C.c_int64), ("stats_ms", C.c_double), ("n_stats", C.c_int64),
                ("dedisperse_bytes", C.c_int64), ("refine_ms", C.c_double), ("n_refine", C.c_int64),
                ("refine_units", C.c_int64)]


CANDIDATE_FIELDS = [f for f, _ in Candidate._fields_ if f != "reserved"]

_P = C.c_void_p
_SIGS = {
    "frbx_version": ([], C.c_char_p),
    "frbx_create": ([C.POINTER(Layout), C.c_int, _P, C.POINTER(_P)], C.c_int),
    "frbx_destroy": ([_P], None),
    "frbx_last_error": ([_P], C.c_char_p),
    "frbx_set_calibration": ([_P, _P, _P], C.c_int),
    "frbx_set_dm_grid": ([_P, C.c_double, C.c_double, C.c_int32, C.c_double], C.c_int),
    "frbx_set_delay_grid": ([_P, C.c_int32, C.c_int32, C.c_double, C.c_double], C.c_int),
    "frbx_set_rate_grid": ([_P, C.c_int32, C.c_double], C.c_int),
    "frbx_set_windows": ([_P, _P, C.c_int32], C.c_int),
    "frbx_set_detection": ([_P, C.c_double, C.c_int32, C.c_int32], C.c_int),
    "frbx_load": ([_P, _P, C.c_int], C.c_int),
    "frbx_load_f16": ([_P, _P, C.c_int], C.c_int),
    "frbx_set_precision": ([_P, C.c_int32], C.c_int),
    "frbx_set_tile_budget": ([_P, C.c_int64], C.c_int),
    "frbx_set_specialisation": ([_P, C.c_int], C.c_int),
    "frbx_set_sbd_matrix_cores": ([_P, C.c_int], C.c_int),
    "frbx_get_specialisation": ([_P, C.POINTER(C.c_uint32), C.POINTER(C.c_char_p)], C.c_int),
    "frbx_run": ([_P], C.c_int),
    "frbx_run_cube_noalloc": ([_P, _P, _P, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "frbx_get_segments": ([_P, _P, _P, _P, _P], C.c_int),
    "frbx_get_lattice": ([_P, _P, _P, _P], C.c_int),
    "frbx_set_recheck": ([_P, C.c_double], C.c_int),
    "frbx_get_recheck": ([_P, _P, _P], C.c_int),
    "frbx_get_ap_offsets": ([_P, _P, C.c_int64, _P], C.c_int),
    "frbx_get_power_cube": ([_P, _P, _P, C.c_int64, _P], C.c_int),
    "frbx_get_power_cube_device": ([_P, _P, _P], C.c_int),
    "frbx_get_stats": ([_P, _P, _P, _P, C.c_int64, _P], C.c_int),
    "frbx_get_crossings": ([_P, _P, C.c_int64, _P], C.c_int),
    "frbx_get_candidates": ([_P, _P, C.c_int64, _P], C.c_int),
    "frbx_get_groups": ([_P, _P, C.c_int64, _P], C.c_int),
    "frbx_dump_segment": ([_P, C.c_int32, C.c_int32, C.c_int32, C.c_int64, _P], C.c_int),
    "frbx_set_timing": ([_P, C.c_int], C.c_int),
    "frbx_stream_begin": ([_P, C.c_int64], C.c_int),
    "frbx_stream_push": ([_P, _P, C.c_int32, _P, C.c_int], C.c_int),
    "frbx_stream_position": ([_P, _P, _P, _P], C.c_int),
    "frbx_load_e4m3": ([_P, _P, _P, C.c_int], C.c_int),
    "frbx_top_peaks": ([_P, C.c_int64, _P, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "frbx_refine_cells": ([_P, _P, _P], C.c_int),
    "frbx_refine_begin": ([_P, _P, C.c_int64, _P], C.c_int),
    "frbx_refine_run": ([_P, C.c_int32], C.c_int),
    "frbx_refine_results": ([_P, _P, _P, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "frbx_refine_forward": ([_P, _P, _P], C.c_int),
    "frbx_refine_backward": ([_P, _P, _P, _P], C.c_int),
    "frbx_refine_curvature": ([_P, _P, _P], C.c_int),
    "frbx_power_sum": ([_P, _P, C.c_int32, _P, C.c_int64, _P], C.c_int),
    "frbx_calibrate": ([_P, C.c_int32, C.c_int64, C.c_int32, _P, _P], C.c_int),
    "frbx_get_timing": ([_P, _P], C.c_int),
    "frbx_mbd_lattice": ([C.POINTER(Layout), C.c_int32, C.c_double, _P, _P, _P], C.c_int),
    "frbx_ap_offsets": ([C.POINTER(Layout), C.c_double, C.c_double, C.c_int32, C.c_double, _P],
                        C.c_int),
    "frbx_detect": ([_P, C.c_int64, C.c_double, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64,
                     _P, _P, C.c_int64, _P], C.c_int),
}


def exported_names():
    return list(_SIGS)


def lib():
    """Load libfrbx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise FrbxError(E_STATE, f"{_LIB_PATH} is missing: build it with "
                                     "`python -m paper_1801_02391_amd.build`")
        L = C.CDLL(_LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def version():
    return lib().frbx_version().decode()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _layout_struct(layout):
    f0 = np.ascontiguousarray(layout["if_freq_mhz"], dtype=np.float64)
    st = Layout(int(layout["n_baselines"]), len(f0), int(layout["n_chan"]), int(layout["n_frames"]),
                float(layout["t_ap_ms"]), float(layout["chan_bw_mhz"]),
                f0.ctypes.data_as(C.POINTER(C.c_double)))
    return st, f0


def records_to_dicts(arr):
    return [{f: (getattr(r, f)) for f in CANDIDATE_FIELDS} for r in arr]


def dicts_to_records(items):
    """Candidate dicts (fields as returned by the getters) -> a ctypes array."""
    arr = (Candidate * max(1, len(items)))()
    for i, c in enumerate(items):
        for f in CANDIDATE_FIELDS:
            if f in c:
                setattr(arr[i], f, c[f])
        if "group_id" not in c:
            arr[i].group_id = -1
    return arr


def ap_offsets(layout, dm_lo, dm_step, n_dm, k_dm=0.0):
    """Host-only Eq. 2 table [D][N][J] from the library (no device needed)."""
    st, f0 = _layout_struct(layout)
    out = np.zeros((n_dm, len(f0), int(layout["n_chan"])), dtype=np.int32)
    s = lib().frbx_ap_offsets(C.byref(st), dm_lo, dm_step, n_dm, k_dm, _ptr(out))
    if s != OK:
        raise FrbxError(s, "frbx_ap_offsets")
    return out


def mbd_lattice(layout, n_mbd, mbd_step_us=0.0):
    """Host-only MBD lattice of a layout (no device needed): the IFs' lattice
    positions, the MBD step (us) and the shift of the compact one-pass form
    of the float32 transform (-1: two-pass form)."""
    st, f0 = _layout_struct(layout)
    q = np.zeros(len(f0), dtype=np.int64)
    step = C.c_double(0.0)
    shift = C.c_int32(0)
    s = lib().frbx_mbd_lattice(C.byref(st), int(n_mbd), float(mbd_step_us), _ptr(q), C.byref(step),
                               C.byref(shift))
    if s != OK:
        raise FrbxError(s, "frbx_mbd_lattice")
    return dict(q=q.tolist(), mbd_step_us=step.value, compact_shift=shift.value)


def detect(crossings, t_amb_us, n_win_min, n_bl_min, use_mbd=True):
    """Host-only grouping (steps b-d, best DM, cross matching) over a list of
    crossing dicts with at least baseline, dm_index, window_len, k0,
    power_norm, mbd_us.  Returns (detections, groups) as lists of dicts."""
    arr = dicts_to_records(crossings)
    nd, ng = C.c_int64(0), C.c_int64(0)
    L = lib()
    s = L.frbx_detect(arr, len(crossings), t_amb_us, n_win_min, n_bl_min, int(bool(use_mbd)),
                      None, 0, C.byref(nd), None, 0, C.byref(ng))
    if s not in (OK, E_RANGE):
        raise FrbxError(s, "frbx_detect")
    dets = (Candidate * max(1, nd.value))()
    grps = (Group * max(1, ng.value))()
    s = L.frbx_detect(arr, len(crossings), t_amb_us, n_win_min, n_bl_min, int(bool(use_mbd)),
                      dets, nd.value, C.byref(nd), grps, ng.value, C.byref(ng))
    if s != OK:
        raise FrbxError(s, "frbx_detect")
    groups = [{f: getattr(grps[i], f) for f, _ in Group._fields_} for i in range(ng.value)]
    return records_to_dicts(dets[:nd.value]), groups


class Search:
    """One search context on one GPU and one HIP stream."""

    def __init__(self, layout, device=0, stream=None):
        import torch  # device memory and streams
        self._torch = torch
        L = lib()
        st, self._f0 = _layout_struct(layout)
        self.layout = dict(layout)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = _P()
        s = L.frbx_create(C.byref(st), int(device), _P(stream.cuda_stream), C.byref(h))
        if s != OK:
            raise FrbxError(s, "frbx_create")
        self._h = h
        self.device = device
        self._vis = None
        self._windows = [2, 4]

    def close(self):
        if getattr(self, "_h", None):
            lib().frbx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, s, what):
        if s != OK:
            msg = lib().frbx_last_error(self._h).decode()
            raise FrbxError(s, f"{what}: {msg}")

    # --------------------------------------------------------------- setup
    def configure(self, search, tau0_us=None, phi0_rad=None):
        """Apply a search-parameter dict (keys of the workload 'search'
        section) and optional calibration [B][N]."""
        L = lib()
        h = self._h
        self._chk(L.frbx_set_dm_grid(h, search["dm_lo"], search["dm_step"], search["n_dm"],
                                     search.get("k_dm", 0.0)), "set_dm_grid")
        f_ref = search.get("f_ref_fit_mhz", float("nan"))
        self._chk(L.frbx_set_delay_grid(h, search["sbd_pad"], search["n_mbd"],
                                        search.get("mbd_step_us", 0.0), f_ref), "set_delay_grid")
        self._chk(L.frbx_set_rate_grid(h, search["n_rate"], search.get("rate_step", 0.0)),
                  "set_rate_grid")
        w = np.ascontiguousarray(search["windows"], dtype=np.int32)
        self._windows = list(map(int, w))
        self._chk(L.frbx_set_windows(h, _ptr(w), len(w)), "set_windows")
        self._chk(L.frbx_set_detection(h, search["threshold"], search["n_win_min"],
                                       search["n_bl_min"]), "set_detection")
        prec = search.get("precision", "f32")
        self._chk(L.frbx_set_precision(h, PRECISIONS[prec] if isinstance(prec, str) else int(prec)),
                  "set_precision")
        self._chk(L.frbx_set_recheck(h, float(search.get("recheck_band", 0.0))), "set_recheck")
        self._chk(L.frbx_set_sbd_matrix_cores(h, 1 if search.get("sbd_mfma", False) else 0), "set_sbd_matrix_cores")
        if tau0_us is not None or phi0_rad is not None:
            t = None if tau0_us is None else np.ascontiguousarray(tau0_us, dtype=np.float64)
            p = None if phi0_rad is None else np.ascontiguousarray(phi0_rad, dtype=np.float64)
            self._chk(L.frbx_set_calibration(h, _ptr(t), _ptr(p)), "set_calibration")
        self.search = dict(search)

    def load(self, vis):
        """vis: [B][N][J][K] complex64, or float16 [B][N][J][K][2] (re, im), as
        a torch tensor (on this device: borrowed) or a numpy array (copied)."""
        torch = self._torch
        if isinstance(vis, torch.Tensor):
            if not vis.is_contiguous() or vis.device.type != "cuda":
                raise FrbxError(E_INVAL, "vis must be a contiguous tensor on the GPU")
            if vis.dtype == torch.complex64:
                fn = lib().frbx_load
            elif vis.dtype == torch.float16 and vis.shape[-1] == 2:
                fn = lib().frbx_load_f16
            else:
                raise FrbxError(E_INVAL, "vis must be complex64 or float16 (re, im) pairs")
            self._vis = vis
            self._chk(fn(self._h, _P(vis.data_ptr()), 1), "load")
        else:
            if vis.dtype == np.float16:
                a = np.ascontiguousarray(vis)
                self._chk(lib().frbx_load_f16(self._h, _ptr(a), 0), "load")
            else:
                a = np.ascontiguousarray(vis, dtype=np.complex64)
                self._chk(lib().frbx_load(self._h, _ptr(a), 0), "load")

    def load_e4m3(self, codes, scale):
        """codes: uint8 [B][N][J][K][2] OCP FP8 e4m3 (re, im); scale: float32
        [B][N][J]; both torch GPU tensors (read during the call) or both numpy
        arrays (copied).  Decoded exactly on the device and searched."""
        torch = self._torch
        if isinstance(codes, torch.Tensor):
            if not (isinstance(scale, torch.Tensor) and codes.device.type == "cuda" and scale.device.type == "cuda"
                    and codes.dtype == torch.uint8 and scale.dtype == torch.float32
                    and codes.is_contiguous() and scale.is_contiguous()):
                raise FrbxError(E_INVAL, "codes (uint8) and scale (float32) must be contiguous GPU tensors")
            self._chk(lib().frbx_load_e4m3(self._h, _P(codes.data_ptr()), _P(scale.data_ptr()), 1), "load_e4m3")
        else:
            c = np.ascontiguousarray(codes, dtype=np.uint8)
            sc = np.ascontiguousarray(scale, dtype=np.float32)
            self._chk(lib().frbx_load_e4m3(self._h, _ptr(c), _ptr(sc), 0), "load_e4m3")
        self._vis = None

    def run(self):
        self._chk(lib().frbx_run(self._h), "run")

    def set_tile_budget(self, n_bytes):
        """Device memory for the dedispersed DM tiles (0: default 6 GiB)."""
        self._chk(lib().frbx_set_tile_budget(self._h, int(n_bytes)), "set_tile_budget")

    def set_specialisation(self, enable):
        """frbx_set_specialisation: float32 fringe kernel compiled for the
        IF lattice's first-pass rows (True, default) or the static one."""
        self._chk(lib().frbx_set_specialisation(self._h, 1 if enable else 0), "set_specialisation")

    def specialisation(self):
        """(row mask of the kernel the last run used, 0 for the static
        kernel; reason it could not be built, or '')."""
        rows = C.c_uint32(0)
        why = C.c_char_p()
        self._chk(lib().frbx_get_specialisation(self._h, C.byref(rows), C.byref(why)), "get_specialisation")
        return int(rows.value), (why.value or b"").decode()

    def run_cube_noalloc(self, power, idx):
        """frbx_run_cube_noalloc into caller-owned contiguous GPU tensors
        (power float32, idx int32, each of B * D * segments elements or
        more); enqueued on the context's stream.  Returns the element count
        written."""
        torch = self._torch
        if not (isinstance(power, torch.Tensor) and isinstance(idx, torch.Tensor)
                and power.device.type == "cuda" and idx.device.type == "cuda"
                and power.dtype == torch.float32 and idx.dtype == torch.int32
                and power.is_contiguous() and idx.is_contiguous()):
            raise FrbxError(E_INVAL, "power (float32) and idx (int32) must be contiguous GPU tensors")
        n = C.c_int64(0)
        self._chk(lib().frbx_run_cube_noalloc(self._h, _P(power.data_ptr()), _P(idx.data_ptr()),
                                              min(power.numel(), idx.numel()), C.byref(n)),
                  "run_cube_noalloc")
        return n.value

    # ------------------------------------------------------------- results
    def segments(self):
        nw = len(self._windows)
        dkm = C.c_int64(0)
        hop = np.zeros(nw, dtype=np.int32)
        nseg = np.zeros(nw, dtype=np.int64)
        tot = C.c_int64(0)
        self._chk(lib().frbx_get_segments(self._h, C.byref(dkm), _ptr(hop), _ptr(nseg),
                                          C.byref(tot)), "get_segments")
        return dict(dk_max=dkm.value, hop=hop.tolist(), n_seg=nseg.tolist(), total=tot.value)

    def recheck(self):
        """(band, segments re-evaluated in float32 by the last run or push: those
        whose normalised power exceeded threshold - band)."""
        band = C.c_double(0.0)
        n = C.c_int64(0)
        self._chk(lib().frbx_get_recheck(self._h, C.byref(band), C.byref(n)), "get_recheck")
        return band.value, n.value

    def lattice(self):
        """MBD lattice positions of the IFs, the MBD step (us) and the shift
        of the compact one-pass form of the float32 transform (-1: general)."""
        q = np.zeros(self.layout["n_if"], dtype=np.int64)
        step = C.c_double(0.0)
        shift = C.c_int32(0)
        self._chk(lib().frbx_get_lattice(self._h, _ptr(q), C.byref(step), C.byref(shift)),
                  "get_lattice")
        return dict(q=q.tolist(), mbd_step_us=step.value, compact_shift=shift.value)

    def ap_offsets(self):
        n = C.c_int64(0)
        L = lib()
        L.frbx_get_ap_offsets(self._h, None, 0, C.byref(n))
        out = np.zeros(n.value, dtype=np.int32)
        self._chk(L.frbx_get_ap_offsets(self._h, _ptr(out), n.value, C.byref(n)), "get_ap_offsets")
        return out.reshape(self.search["n_dm"], self.layout["n_if"] if "n_if" in self.layout
                           else len(self._f0), self.layout["n_chan"])

    def power_cube(self):
        """(power [B][D][S] float32, packed index [B][D][S] int32) on the host."""
        n = C.c_int64(0)
        L = lib()
        s = L.frbx_get_power_cube(self._h, None, None, 0, C.byref(n))
        if s not in (OK, E_RANGE):
            self._chk(s, "get_power_cube")
        p = np.zeros(n.value, dtype=np.float32)
        i = np.zeros(n.value, dtype=np.int32)
        self._chk(L.frbx_get_power_cube(self._h, _ptr(p), _ptr(i), n.value, C.byref(n)),
                  "get_power_cube")
        B, D = self.layout["n_baselines"], self.search["n_dm"]
        return p.reshape(B, D, -1), i.reshape(B, D, -1)

    def stats(self):
        n = C.c_int64(0)
        L = lib()
        L.frbx_get_stats(self._h, None, None, None, 0, C.byref(n))
        m = np.zeros(n.value)
        s = np.zeros(n.value)
        c = np.zeros(n.value, dtype=np.int64)
        self._chk(L.frbx_get_stats(self._h, _ptr(m), _ptr(s), _ptr(c), n.value, C.byref(n)),
                  "get_stats")
        return m, s, c

    def _records(self, fn, what):
        n = C.c_int64(0)
        s = fn(self._h, None, 0, C.byref(n))
        if s not in (OK, E_RANGE):
            self._chk(s, what)
        arr = (Candidate * max(1, n.value))()
        self._chk(fn(self._h, arr, n.value, C.byref(n)), what)
        return records_to_dicts(arr[:n.value])

    def crossings(self):
        return self._records(lib().frbx_get_crossings, "get_crossings")

    def candidates(self):
        return self._records(lib().frbx_get_candidates, "get_candidates")

    def groups(self):
        L = lib()
        n = C.c_int64(0)
        s = L.frbx_get_groups(self._h, None, 0, C.byref(n))
        if s not in (OK, E_RANGE):
            self._chk(s, "get_groups")
        arr = (Group * max(1, n.value))()
        self._chk(L.frbx_get_groups(self._h, arr, n.value, C.byref(n)), "get_groups")
        return [{f: getattr(arr[i], f) for f, _ in Group._fields_} for i in range(n.value)]

    # ------------------------------------------------------------ streaming
    _KINDS = {"c64": 0, "c32": 1, "e4m3": 2}

    def stream_begin(self, chunk_frames):
        self._chk(lib().frbx_stream_begin(self._h, int(chunk_frames)), "stream_begin")

    def stream_push(self, chunk, kind="c64", scale=None):
        """chunk: [B][N][J][chunk] complex64, float16 [..][2] (c32) or uint8
        [..][2] (e4m3, with float32 scale [B][N][J]); torch (device) or numpy."""
        torch = self._torch
        k = self._KINDS[kind]
        if isinstance(chunk, torch.Tensor):
            if not chunk.is_contiguous() or chunk.device.type != "cuda":
                raise FrbxError(E_INVAL, "chunk must be a contiguous GPU tensor")
            sp = None
            if k == 2:
                if not isinstance(scale, torch.Tensor) or scale.dtype != torch.float32:
                    raise FrbxError(E_INVAL, "e4m3 chunks need a float32 scale tensor")
                sp = _P(scale.contiguous().data_ptr())
            self._chk(lib().frbx_stream_push(self._h, _P(chunk.data_ptr()), k, sp, 1), "stream_push")
        else:
            a = np.ascontiguousarray(chunk)
            sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float32)
            self._chk(lib().frbx_stream_push(self._h, _ptr(a), k, _ptr(sc), 0), "stream_push")

    def stream_position(self):
        nw = len(self._windows)
        fi = C.c_int64(0)
        first = np.zeros(nw, dtype=np.int64)
        nseg = np.zeros(nw, dtype=np.int64)
        self._chk(lib().frbx_stream_position(self._h, C.byref(fi), _ptr(first), _ptr(nseg)),
                  "stream_position")
        return dict(frames_in=fi.value, first=first.tolist(), n_seg=nseg.tolist())

    def power_sum(self, baselines):
        """Sec. 2.4.2 detections from the summed power of `baselines`."""
        bl = np.ascontiguousarray(baselines, dtype=np.int32)
        L = lib()
        n = C.c_int64(0)
        s = L.frbx_power_sum(self._h, _ptr(bl), len(bl), None, 0, C.byref(n))
        if s not in (OK, E_RANGE):
            self._chk(s, "power_sum")
        arr = (Candidate * max(1, n.value))()
        self._chk(L.frbx_power_sum(self._h, _ptr(bl), len(bl), arr, n.value, C.byref(n)),
                  "power_sum")
        return records_to_dicts(arr[:n.value])

    def calibrate(self, baseline, k0, length):
        """Appendix A extraction on a calibrator segment -> (tau0_us[N], phi0_rad[N])."""
        N = len(self._f0)
        t = np.zeros(N)
        p = np.zeros(N)
        self._chk(lib().frbx_calibrate(self._h, int(baseline), int(k0), int(length), _ptr(t), _ptr(p)),
                  "calibrate")
        return t, p

    # ----------------------------------------------------------- refinement
    REFINE_PARAMS = ("sbd_us", "mbd_us", "rate", "dm", "t_frames")

    def top_peaks(self, n_max):
        """The n_max crossings of the last run with the highest normalised power."""
        L = lib()
        n = C.c_int64(0)
        s = L.frbx_top_peaks(self._h, int(n_max), None, 0, C.byref(n))
        if s not in (OK, E_RANGE):
            self._chk(s, "top_peaks")
        arr = (Candidate * max(1, n.value))()
        self._chk(L.frbx_top_peaks(self._h, int(n_max), arr, n.value, C.byref(n)), "top_peaks")
        return records_to_dicts(arr[:n.value])

    def refine_cells(self):
        cells = np.zeros(5)
        xbar = C.c_double(0.0)
        self._chk(lib().frbx_refine_cells(self._h, _ptr(cells), C.byref(xbar)), "refine_cells")
        return cells, xbar.value

    def refine_begin(self, peaks):
        """Start a refinement of the given candidate records (dicts or
        Candidate records); returns the start parameters [n][5]."""
        recs = dicts_to_records(peaks)
        n = len(peaks)
        th0 = np.zeros((max(n, 1), 5))
        self._chk(lib().frbx_refine_begin(self._h, recs, n, _ptr(th0)), "refine_begin")
        self._refine_n = n
        return th0[:n]

    def refine(self, peaks, steps=20):
        """The library's ascent: (start theta [n][5], final theta [n][5], final |G| [n])."""
        th0 = self.refine_begin(peaks)
        self._chk(lib().frbx_refine_run(self._h, int(steps)), "refine_run")
        n = C.c_int64(0)
        th = np.zeros((max(len(peaks), 1), 5))
        p = np.zeros(max(len(peaks), 1), dtype=np.float32)
        self._chk(lib().frbx_refine_results(self._h, _ptr(th), _ptr(p), len(peaks), C.byref(n)),
                  "refine_results")
        return th0, th[:n.value], p[:n.value]

    def _dev(self, t, dtype, shape):
        torch = self._torch
        if (not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device.type != "cuda"
                or not t.is_contiguous() or tuple(t.shape) != tuple(shape)):
            raise FrbxError(E_INVAL, f"expected a contiguous {dtype} GPU tensor of shape {shape}")
        return _P(t.data_ptr())

    def refine_forward(self, theta):
        """|G| at theta [n][5] (float64 GPU tensor) of the begun peaks."""
        torch = self._torch
        n = self._refine_n
        out = torch.empty(n, dtype=torch.float32, device=theta.device)
        self._chk(lib().frbx_refine_forward(self._h, self._dev(theta, torch.float64, (n, 5)),
                                            self._dev(out, torch.float32, (n,))), "refine_forward")
        return out

    def refine_backward(self, theta, grad_power):
        torch = self._torch
        n = self._refine_n
        g = torch.empty((n, 5), dtype=torch.float64, device=theta.device)
        self._chk(lib().frbx_refine_backward(self._h, self._dev(theta, torch.float64, (n, 5)),
                                             self._dev(grad_power, torch.float32, (n,)),
                                             self._dev(g, torch.float64, (n, 5))), "refine_backward")
        return g

    def refine_curvature(self, theta):
        torch = self._torch
        n = self._refine_n
        h = torch.empty((n, 6), dtype=torch.float64, device=theta.device)
        self._chk(lib().frbx_refine_curvature(self._h, self._dev(theta, torch.float64, (n, 5)),
                                              self._dev(h, torch.float64, (n, 6))), "refine_curvature")
        return h

    def set_timing(self, enable=True):
        self._chk(lib().frbx_set_timing(self._h, int(bool(enable))), "set_timing")

    def timing(self):
        t = Timing()
        self._chk(lib().frbx_get_timing(self._h, C.byref(t)), "get_timing")
        return {f: getattr(t, f) for f, _ in Timing._fields_}

    def dump_segment(self, b, d, wi, q):
        """|G|^2 of every (rate, SBD, MBD) cell of one segment -> numpy [R][PJ][M]."""
        torch = self._torch
        R = self.search["n_rate"]
        PJ = self.search["sbd_pad"] * self.layout["n_chan"]
        M = self.search["n_mbd"]
        out = torch.empty(R * PJ * M, dtype=torch.float32, device=f"cuda:{self.device}")
        self._chk(lib().frbx_dump_segment(self._h, b, d, wi, q, _P(out.data_ptr())),
                  "dump_segment")
        return out.cpu().numpy().reshape(R, PJ, M)


def _refine_function():
    import torch

    class RefinePower(torch.autograd.Function):
        """P = |G|(theta) of the begun peaks: forward and backward are the
        library's refinement kernels (float32 sums, float64 phases)."""

        @staticmethod
        def forward(ctx, theta, search):
            th = theta.detach().contiguous()
            ctx.save_for_backward(th)
            ctx.search = search
            return search.refine_forward(th)

        @staticmethod
        def backward(ctx, grad_power):
            (th,) = ctx.saved_tensors
            g = ctx.search.refine_backward(th, grad_power.detach().to(torch.float32).contiguous())
            return g, None

    return RefinePower


_REFINE_FN = None


def refine_power(theta, search):
    """torch.autograd entry: |G| [n] of the peaks begun on `search` at
    theta [n][5] (float64 GPU tensor, requires_grad allowed)."""
    global _REFINE_FN
    if _REFINE_FN is None:
        _REFINE_FN = _refine_function()
    return _REFINE_FN.apply(theta, search)
