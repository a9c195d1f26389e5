"""Python face of the Power-ψ library: the C-ABI calls under the same names.

PyTorch supplies device memory (workspaces and result tensors are torch
tensors) and the stream; every step of the computation runs in the HIP
kernels of libpsi.so.  Nothing here computes ψ.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _ffi
from ._ffi import (PSI_INPUT_HOST, PSI_NO_FALLBACK, PSI_PREC_FP32,  # noqa: F401
                   PSI_PREC_FP64, PSI_PREC_FP64_WEIGHTED, PSI_PREC_MIXED, PSI_STRICT,
                   PSI_TOL_ABS_L1, PSI_TOL_BNORM, PSI_TOL_REL_L1, PSI_WEIGHTED_FP64)

PRECISIONS = {"fp64": PSI_PREC_FP64, "fp64_weighted": PSI_PREC_FP64_WEIGHTED,
              "mixed": PSI_PREC_MIXED, "fp32": PSI_PREC_FP32}
TOL_MODES = {"abs_l1": PSI_TOL_ABS_L1, "bnorm": PSI_TOL_BNORM, "rel_l1": PSI_TOL_REL_L1}
SEG_FORMS = {"auto": 0, "none": 0, "tiles": _ffi.PSI_SEG_TILES, "slices": _ffi.PSI_SEG_SLICES,
             "bands": _ffi.PSI_SEG_BANDS, "bins": _ffi.PSI_SEG_BINS}
SEG_FORM_NAMES = {0: "none", _ffi.PSI_SEG_TILES: "tiles", _ffi.PSI_SEG_SLICES: "slices",
                  _ffi.PSI_SEG_BANDS: "bands", _ffi.PSI_SEG_BINS: "bins"}


def _seg_form(f) -> int:
    return SEG_FORMS[f] if isinstance(f, str) else int(f)


class PsiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_ffi.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load():
    return _ffi.load()


def _check(status: int):
    if status != _ffi.PSI_OK:
        raise PsiError(status, _ffi.load().psi_last_error().decode())


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _device(device) -> torch.device:
    """A CUDA device with its index (the current device when none is given)."""
    d = torch.device(device) if device is not None else torch.device("cuda")
    if d.type != "cuda":
        raise ValueError(f"the library runs on a GPU, not on {d}")
    return d if d.index is not None else torch.device("cuda", torch.cuda.current_device())


def _vec_in(t, n: int, device: torch.device, dtype: torch.dtype, name: str) -> torch.Tensor:
    """An input vector as a contiguous device tensor of exactly n values: the
    kernels read n entries from its pointer, so a shorter one is refused."""
    t = torch.as_tensor(t).to(device, dtype).contiguous()
    if t.numel() != n:
        raise ValueError(f"{name} must hold {n} values, not {t.numel()}")
    return t


def _vec_out(t, n: int, device: torch.device, dtype: torch.dtype, name: str) -> torch.Tensor:
    """A result buffer: a new one, or the caller's if it is a contiguous
    tensor of n values of the right type on the operator's device."""
    if t is None:
        return torch.empty(n, dtype=dtype, device=device)
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or \
            not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {n} values on {device}")
    return t


def version() -> str:
    return _ffi.load().psi_version().decode()


def workspace_size(n_users: int, n_edges: int, n_graphs: int = 1, flags: int = 0) -> tuple[int, int]:
    lib = _ffi.load()
    p, s = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.psi_operator_workspace_size(n_users, n_edges, n_graphs, flags, ctypes.byref(p),
                                           ctypes.byref(s)))
    return p.value, s.value


class Operator:
    """A built Power-ψ operator (psi_build_operator) and its device workspace.

    follower/leader/lam/mu are numpy arrays (passed as host memory) or CUDA
    torch tensors (int32 / float64).  Edge k means follower[k] follows
    leader[k].
    """

    def __init__(self, n_users, follower, leader, lam, mu, node_offsets=None, flags: int = 0,
                 stream=None, device=None):
        lib = _ffi.load()
        self._lib = lib
        self.device = _device(device)
        host = isinstance(follower, np.ndarray)
        keep = []
        if host:
            f = np.ascontiguousarray(follower, dtype=np.int32)
            l = np.ascontiguousarray(leader, dtype=np.int32)
            la = np.ascontiguousarray(lam, dtype=np.float64)
            m_ = np.ascontiguousarray(mu, dtype=np.float64)
            keep = [f, l, la, m_]
            ptrs = [a.ctypes.data for a in keep]
            flags |= PSI_INPUT_HOST
            n_edges = int(f.shape[0])
        else:
            f = torch.as_tensor(follower).to(self.device, torch.int32).contiguous()
            l = torch.as_tensor(leader).to(self.device, torch.int32).contiguous()
            la = torch.as_tensor(lam).to(self.device, torch.float64).contiguous()
            m_ = torch.as_tensor(mu).to(self.device, torch.float64).contiguous()
            keep = [f, l, la, m_]
            ptrs = [a.data_ptr() for a in keep]
            n_edges = int(f.shape[0])
        # the build reads n_edges pairs and n_users activities from these pointers
        if f.ndim != 1 or l.shape != f.shape:
            raise ValueError("follower and leader must be 1-D arrays of the same length")
        if la.shape != (int(n_users),) or m_.shape != (int(n_users),):
            raise ValueError(f"lam and mu must each hold n_users = {int(n_users)} values")
        n_graphs = 1
        offs_ptr = None
        if node_offsets is not None:
            offs = np.ascontiguousarray(node_offsets, dtype=np.int64)
            if offs.ndim != 1 or offs.size < 2:
                raise ValueError("node_offsets must be a 1-D array of n_graphs + 1 offsets")
            n_graphs = int(offs.shape[0] - 1)
            keep.append(offs)
            offs_ptr = offs.ctypes.data
            self.node_offsets = offs.copy()
        else:
            self.node_offsets = np.array([0, n_users], dtype=np.int64)
        self.n = int(n_users)
        self.n_graphs = n_graphs
        self.flags = flags
        pbytes, sbytes = workspace_size(self.n, n_edges, n_graphs, flags)
        self.workspace = torch.empty(pbytes, dtype=torch.uint8, device=self.device)
        scratch = torch.empty(sbytes, dtype=torch.uint8, device=self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = _stream_handle(stream)
            _check(lib.psi_build_operator(self.n, n_edges, ptrs[0], ptrs[1], ptrs[2], ptrs[3],
                                          n_graphs, offs_ptr, flags, self.workspace.data_ptr(),
                                          pbytes, scratch.data_ptr(), sbytes, st,
                                          ctypes.byref(handle)))
        del scratch
        self._h = handle

    # ------------------------------------------------------------------ queries
    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = _ffi.OperatorStats()
        _check(self._lib.psi_operator_get_stats(self._h, ctypes.byref(s)))
        return _ffi.struct_dict(s)

    def views(self) -> dict:
        """row_ptr, col, c, d, inv_den as tensors aliasing the workspace."""
        ptrs = [ctypes.c_void_p() for _ in range(5)]
        _check(self._lib.psi_operator_views(self._h, *[ctypes.byref(p) for p in ptrs]))
        st = self.stats()
        base = self.workspace.data_ptr()
        out = {}
        for name, p, dt, cnt in (("row_ptr", ptrs[0], torch.int32, self.n + 1),
                                 ("col", ptrs[1], torch.int32, st["n_edges"]),
                                 ("c", ptrs[2], torch.float64, self.n),
                                 ("d", ptrs[3], torch.float64, self.n),
                                 ("inv_den", ptrs[4], torch.float64, self.n)):
            off = p.value - base
            nbytes = cnt * torch.tensor([], dtype=dt).element_size()
            out[name] = self.workspace[off:off + nbytes].view(dt)
        return out

    def bins_info(self) -> dict:
        """psi_operator_bins_info: the binned layout built on the operator."""
        v = [ctypes.c_int32() for _ in range(5)] + [ctypes.c_int64()]
        _check(self._lib.psi_operator_bins_info(self._h, *[ctypes.byref(x) for x in v]))
        keys = ("block_users", "rows", "col_blocks", "bins", "split_rows", "runs")
        return {k: x.value for k, x in zip(keys, v)}

    def band_info(self) -> dict:
        """psi_operator_band_info: the band layout built on the operator."""
        v = [ctypes.c_int32() for _ in range(6)]
        _check(self._lib.psi_operator_band_info(self._h, *[ctypes.byref(x) for x in v]))
        keys = ("col_log", "rows", "col_blocks", "row_blocks", "bands", "split_rows")
        return {k: x.value for k, x in zip(keys, v)}

    def debug_force_slot_timeout(self, on: bool) -> None:
        """psi_debug_force_slot_timeout: make every bounded wait of this
        operator's passes give up at once (tests of the recovery path)."""
        _check(self._lib.psi_debug_force_slot_timeout(self._h, 1 if on else 0))

    # ------------------------------------------------------------------ compute
    def solve(self, tol: float = 1e-8, tol_mode: str = "abs_l1", max_iter: int = 10000,
              precision: str = "fp64", s0: torch.Tensor | None = None, check_every: int = 0,
              tile_items: int = 0, col_segments: int = 0, inner_tol: float = 0.0,
              no_fallback: bool = False, seg_form: str | int = 0,
              return_s: bool = False, psi_out: torch.Tensor | None = None, stream=None,
              raise_on_status: bool = False, band_col_log: int = 0, band_rows: int = 0):
        """psi_solve: ψ (and s) by Algorithm 2; returns (psi, info) or (psi, s, info).
        seg_form: 0 / "auto", "tiles" or "slices" (partial pass of a segmented
        pass), "bands" (column-blocked layout with band_col_log, band_rows) or
        "bins" (binned two-launch pass)."""
        p = _ffi.Params()
        _check(self._lib.psi_params_default(ctypes.byref(p)))
        p.tol = tol
        p.tol_mode = TOL_MODES[tol_mode] if isinstance(tol_mode, str) else int(tol_mode)
        p.max_iter = max_iter
        p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        p.check_every = check_every
        p.flags = PSI_NO_FALLBACK if no_fallback else 0
        p.tile_items = tile_items
        p.col_segments = col_segments
        p.seg_form = _seg_form(seg_form)
        p.inner_tol = inner_tol
        p.band_col_log = band_col_log
        p.band_rows = band_rows
        psi = _vec_out(psi_out, self.n, self.device, torch.float64, "psi_out")
        s = torch.empty(self.n, dtype=torch.float64, device=self.device) if return_s else None
        if s0 is not None:
            s0 = _vec_in(s0, self.n, self.device, torch.float64, "s0")
        info = _ffi.Info()
        with torch.cuda.device(self.device):
            st = self._lib.psi_solve(self._h, ctypes.byref(p), _ptr(s0), _ptr(psi), _ptr(s),
                                     ctypes.byref(info), _stream_handle(stream))
        d = _ffi.struct_dict(info)
        d["status_name"] = _ffi.STATUS_NAMES.get(st, str(st))
        if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE) or (
                raise_on_status and st != _ffi.PSI_OK):
            _check(st)
        return (psi, s, d) if return_s else (psi, d)

    def solve_async(self, tol: float = 1e-8, tol_mode: str = "abs_l1", max_iter: int = 10000,
                    s0: torch.Tensor | None = None, check_every: int = 0,
                    band_col_log: int = 0, band_rows: int = 0, return_s: bool = False,
                    stream=None, raise_on_status: bool = False):
        """psi_solve_async: the same ψ by block Gauss–Seidel sweeps over the band
        layout; returns (psi, info) or (psi, s, info)."""
        p = _ffi.Params()
        _check(self._lib.psi_params_default(ctypes.byref(p)))
        p.tol = tol
        p.tol_mode = TOL_MODES[tol_mode] if isinstance(tol_mode, str) else int(tol_mode)
        p.max_iter = max_iter
        p.check_every = check_every
        p.band_col_log = band_col_log
        p.band_rows = band_rows
        psi = torch.empty(self.n, dtype=torch.float64, device=self.device)
        s = torch.empty(self.n, dtype=torch.float64, device=self.device) if return_s else None
        if s0 is not None:
            s0 = _vec_in(s0, self.n, self.device, torch.float64, "s0")
        info = _ffi.Info()
        with torch.cuda.device(self.device):
            st = self._lib.psi_solve_async(self._h, ctypes.byref(p), _ptr(s0), _ptr(psi), _ptr(s),
                                           ctypes.byref(info), _stream_handle(stream))
        d = _ffi.struct_dict(info)
        d["status_name"] = _ffi.STATUS_NAMES.get(st, str(st))
        if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE) or (
                raise_on_status and st != _ffi.PSI_OK):
            _check(st)
        return (psi, s, d) if return_s else (psi, d)

    def step(self, s_in: torch.Tensor, precision: str = "fp64", tile_items: int = 0,
             col_segments: int = 0, seg_form: str | int = 0, stream=None):
        """psi_step: one Power-ψ step s_out = Aᵀ s_in + c and its L1 gap (enqueued)."""
        s_in = _vec_in(s_in, self.n, self.device, torch.float64, "s_in")
        out = torch.empty_like(s_in)
        gap = torch.empty(1, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(self._lib.psi_step(self._h, PRECISIONS[precision], s_in.data_ptr(),
                                      out.data_ptr(), gap.data_ptr(), tile_items,
                                      col_segments, _seg_form(seg_form),
                                      _stream_handle(stream)))
        return out, gap

    def final(self, s: torch.Tensor, stream=None) -> torch.Tensor:
        """psi_final: ψ = (Bᵀ s + d)/N (enqueued)."""
        s = _vec_in(s, self.n, self.device, torch.float64, "s")
        out = torch.empty_like(s)
        with torch.cuda.device(self.device):
            _check(self._lib.psi_final(self._h, s.data_ptr(), out.data_ptr(),
                                       _stream_handle(stream)))
        return out

    def pass_time(self, kind: str, reps: int = 50, tile_items: int = 0, col_segments: int = 0,
                  seg_form: str | int = 0, stream=None) -> float:
        """psi_pass_time: mean ms of one launch of a pass kind (HIP events on the stream)."""
        kinds = {"step64": _ffi.PSI_PASS_STEP64, "step64_w": _ffi.PSI_PASS_STEP64_W,
                 "final64": _ffi.PSI_PASS_FINAL64, "step32": _ffi.PSI_PASS_STEP32,
                 "part64": _ffi.PSI_PASS_PART64, "part32": _ffi.PSI_PASS_PART32}
        out = ctypes.c_double()
        with torch.cuda.device(self.device):
            _check(self._lib.psi_pass_time(self._h, kinds[kind], reps, tile_items, col_segments,
                                           _seg_form(seg_form), ctypes.byref(out),
                                           _stream_handle(stream)))
        return out.value

    def autotune(self, precision: str = "fp64", reps: int = 0, stream=None) -> dict:
        """psi_autotune: the fastest tile_items / col_segments / seg_form for
        `precision`, kept in the operator for later solves."""
        t, sg, fm, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        with torch.cuda.device(self.device):
            _check(self._lib.psi_autotune(self._h, prec, reps, ctypes.byref(t), ctypes.byref(sg),
                                          ctypes.byref(fm), ctypes.byref(ms),
                                          _stream_handle(stream)))
        return dict(tile_items=t.value, col_segments=sg.value, seg_form=SEG_FORM_NAMES[fm.value],
                    pass_ms=ms.value)

    def _params(self, tol, tol_mode, max_iter, precision, check_every, tile_items=0,
                col_segments=0, inner_tol=0.0, no_fallback=False, seg_form=0):
        p = _ffi.Params()
        _check(self._lib.psi_params_default(ctypes.byref(p)))
        p.tol = tol
        p.tol_mode = TOL_MODES[tol_mode] if isinstance(tol_mode, str) else int(tol_mode)
        p.max_iter = max_iter
        p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        p.check_every = check_every
        p.flags = PSI_NO_FALLBACK if no_fallback else 0
        p.tile_items = tile_items
        p.col_segments = col_segments
        p.seg_form = _seg_form(seg_form)
        p.inner_tol = inner_tol
        return p

    def batched_workspace(self, n_scenarios: int, precision: str = "fp64") -> torch.Tensor:
        """A device workspace of psi_batched_workspace_size bytes (kept and
        reused while large enough)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        nbytes = ctypes.c_size_t()
        _check(self._lib.psi_batched_workspace_size(self._h, int(n_scenarios), prec,
                                                    ctypes.byref(nbytes)))
        ws = getattr(self, "_batch_ws", None)
        if ws is None or ws.numel() < nbytes.value:
            ws = None
            self._batch_ws = None
            ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self._batch_ws = ws
        return ws

    def autotune_batched(self, n_scenarios: int, precision: str = "fp64", reps: int = 0,
                         stream=None) -> dict:
        """psi_autotune_batched: the fastest scenarios per tile / items per wave
        tile / hub chunk for K = n_scenarios, kept for later batched solves."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        ws = self.batched_workspace(n_scenarios, precision)
        bt, bi, bc, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        with torch.cuda.device(self.device):
            _check(self._lib.psi_autotune_batched(self._h, prec, int(n_scenarios), ws.data_ptr(),
                                                  ws.numel(), reps, ctypes.byref(bt),
                                                  ctypes.byref(bi), ctypes.byref(bc),
                                                  ctypes.byref(ms), _stream_handle(stream)))
        return dict(batch_tile=bt.value, batch_items=bi.value, hub_chunk=bc.value,
                    pass_ms=ms.value)

    def autotune_graphs(self, precision: str = "fp64", tol: float = 1e-8, reps: int = 0,
                        stream=None) -> dict:
        """psi_autotune_graphs: the tile_items / col_segments / seg_form whose
        whole graph batch to `tol` is fastest, kept for later graph solves."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        t, sg, fm, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        with torch.cuda.device(self.device):
            _check(self._lib.psi_autotune_graphs(self._h, prec, float(tol), reps, ctypes.byref(t),
                                                 ctypes.byref(sg), ctypes.byref(fm),
                                                 ctypes.byref(ms), _stream_handle(stream)))
        return dict(tile_items=t.value, col_segments=sg.value, seg_form=SEG_FORM_NAMES[fm.value],
                    solve_ms=ms.value)

    def solve_batched(self, lam: torch.Tensor, mu: torch.Tensor, tol: float = 1e-8,
                      max_iter: int = 10000, check_every: int = 0, precision: str = "fp64",
                      inner_tol: float = 0.0, batch_tile: int = 0, batch_items: int = 0,
                      hub_chunk: int = 0, stream=None, raise_on_status: bool = False):
        """psi_solve_batched, scenario mode: lam, mu [N × K] (one column per
        scenario); precision "fp64" or "mixed" (FP32 corrections refined in
        FP64); batch_tile / batch_items / hub_chunk pick the schedule (0 =
        tuned or default); returns (psi [N × K], list of K info dicts)."""
        lam = lam.to(self.device, torch.float64).contiguous()
        mu = mu.to(self.device, torch.float64).contiguous()
        if lam.dim() != 2 or lam.shape != mu.shape or lam.shape[0] != self.n:
            raise ValueError("lam and mu must both be [n_users, n_scenarios]")
        k = int(lam.shape[1])
        p = self._params(tol, "abs_l1", max_iter, precision, check_every, inner_tol=inner_tol)
        p.batch_tile = batch_tile
        p.batch_items = batch_items
        p.hub_chunk = hub_chunk
        nbytes = ctypes.c_size_t()
        _check(self._lib.psi_batched_workspace_size(self._h, k, p.precision, ctypes.byref(nbytes)))
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        psi = torch.empty((self.n, k), dtype=torch.float64, device=self.device)
        infos = (_ffi.Info * k)()
        with torch.cuda.device(self.device):
            st = self._lib.psi_solve_batched(self._h, ctypes.byref(p), k, lam.data_ptr(),
                                             mu.data_ptr(), psi.data_ptr(), infos, ws.data_ptr(),
                                             nbytes.value, _stream_handle(stream))
        if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE) or (
                raise_on_status and st != _ffi.PSI_OK):
            _check(st)
        out = []
        for i in range(k):
            d = _ffi.struct_dict(infos[i])
            d["status_name"] = _ffi.STATUS_NAMES.get(d["status"], str(d["status"]))
            out.append(d)
        return psi, out

    def solve_anderson(self, tol: float = 1e-8, depth: int = 4, tol_mode: str = "abs_l1",
                       max_iter: int = 10000, s0: torch.Tensor | None = None,
                       check_every: int = 0, tile_items: int = 0, col_segments: int = 0,
                       seg_form: str | int = 0, precision: str = "fp64",
                       inner_tol: float = 0.0,
                       return_s: bool = False, stream=None, raise_on_status: bool = False):
        """psi_solve_anderson: the same ψ with Anderson-accelerated passes
        (precision "fp64", or "mixed": accelerated FP32 correction solves
        between FP64 residual passes); returns (psi, info) or (psi, s, info)."""
        p = self._params(tol, tol_mode, max_iter, precision, check_every, tile_items,
                         col_segments, inner_tol=inner_tol, seg_form=seg_form)
        nbytes = ctypes.c_size_t()
        _check(self._lib.psi_anderson_workspace_size(self._h, depth, ctypes.byref(nbytes)))
        ws = self._accel_ws if getattr(self, "_accel_ws", None) is not None and \
            self._accel_ws.numel() >= nbytes.value else None
        if ws is None:
            ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self._accel_ws = ws
        psi = torch.empty(self.n, dtype=torch.float64, device=self.device)
        s = torch.empty(self.n, dtype=torch.float64, device=self.device) if return_s else None
        if s0 is not None:
            s0 = _vec_in(s0, self.n, self.device, torch.float64, "s0")
        info = _ffi.Info()
        with torch.cuda.device(self.device):
            st = self._lib.psi_solve_anderson(self._h, ctypes.byref(p), depth, _ptr(s0),
                                              psi.data_ptr(), _ptr(s), ctypes.byref(info),
                                              ws.data_ptr(), ws.numel(), _stream_handle(stream))
        d = _ffi.struct_dict(info)
        d["status_name"] = _ffi.STATUS_NAMES.get(st, str(st))
        if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE) or (
                raise_on_status and st != _ffi.PSI_OK):
            _check(st)
        return (psi, s, d) if return_s else (psi, d)

    def solve_anderson_noalloc(self, tol: float = 1e-8, depth: int = 4, tol_mode: str = "abs_l1",
                               max_iter: int = 10000, s0: torch.Tensor | None = None,
                               check_every: int = 0, tile_items: int = 0, col_segments: int = 0,
                               seg_form: str | int = 0, precision: str = "fp64",
                               inner_tol: float = 0.0, return_s: bool = False, stream=None,
                               raise_on_status: bool = False):
        """psi_solve_anderson_noalloc: psi_solve_anderson with its scratch in the
        library's fixed device array (no workspace, no device allocation)."""
        p = self._params(tol, tol_mode, max_iter, precision, check_every, tile_items,
                         col_segments, inner_tol=inner_tol, seg_form=seg_form)
        psi = torch.empty(self.n, dtype=torch.float64, device=self.device)
        s = torch.empty(self.n, dtype=torch.float64, device=self.device) if return_s else None
        if s0 is not None:
            s0 = _vec_in(s0, self.n, self.device, torch.float64, "s0")
        info = _ffi.Info()
        with torch.cuda.device(self.device):
            st = self._lib.psi_solve_anderson_noalloc(self._h, ctypes.byref(p), depth, _ptr(s0),
                                                      psi.data_ptr(), _ptr(s), ctypes.byref(info),
                                                      _stream_handle(stream))
        d = _ffi.struct_dict(info)
        d["status_name"] = _ffi.STATUS_NAMES.get(st, str(st))
        if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE) or (
                raise_on_status and st != _ffi.PSI_OK):
            _check(st)
        return (psi, s, d) if return_s else (psi, d)

    def solve_origins(self, origins, tol: float = 1e-8, max_iter: int = 10000,
                      want_p: bool = True, check_every: int = 0, stream=None,
                      raise_on_status: bool = False):
        """psi_solve_origins: Power-NF for the given origin users at once.
        Returns (psi [K], p [N × K] or None, list of K info dicts); column k
        of p is the newsfeed share vector p_i of origin i = origins[k]."""
        org = np.ascontiguousarray(origins, dtype=np.int32)
        if org.ndim != 1 or org.size == 0:
            raise ValueError("origins must be a non-empty 1-D array of user ids")
        k = int(org.size)
        p = self._params(tol, "abs_l1", max_iter, "fp64", check_every)
        nbytes = ctypes.c_size_t()
        _check(self._lib.psi_batched_workspace_size(self._h, k, PSI_PREC_FP64,
                                                    ctypes.byref(nbytes)))
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        psi = torch.empty(k, dtype=torch.float64, device=self.device)
        pm = torch.empty((self.n, k), dtype=torch.float64, device=self.device) if want_p else None
        infos = (_ffi.Info * k)()
        with torch.cuda.device(self.device):
            st = self._lib.psi_solve_origins(self._h, ctypes.byref(p), k, org.ctypes.data,
                                             _ptr(pm), psi.data_ptr(), infos, ws.data_ptr(),
                                             nbytes.value, _stream_handle(stream))
        if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE) or (
                raise_on_status and st != _ffi.PSI_OK):
            _check(st)
        out = []
        for i in range(k):
            d = _ffi.struct_dict(infos[i])
            d["status_name"] = _ffi.STATUS_NAMES.get(d["status"], str(d["status"]))
            out.append(d)
        return psi, pm, out

    def solve_graphs(self, tol: float = 1e-8, max_iter: int = 10000, check_every: int = 0,
                     tile_items: int = 0, col_segments: int = 0, seg_form: str | int = 0,
                     precision: str = "fp64", inner_tol: float = 0.0,
                     stream=None, raise_on_status: bool = False):
        """psi_solve_batched, graph mode: every graph of a block-diagonal
        operator solved to its own tolerance; returns (psi [N], G info dicts).
        col_segments > 1 runs each pass as a column-segmented partial pass
        (seg_form "tiles" or "slices") and a combine; precision "fp64" or
        "mixed" (FP32 corrections refined in FP64, per graph)."""
        if self.n_graphs < 2:
            raise ValueError("graph mode needs an operator built with node_offsets")
        p = self._params(tol, "abs_l1", max_iter, precision, check_every, tile_items,
                         col_segments, inner_tol=inner_tol, seg_form=seg_form)
        psi = torch.empty(self.n, dtype=torch.float64, device=self.device)
        infos = (_ffi.Info * self.n_graphs)()
        with torch.cuda.device(self.device):
            st = self._lib.psi_solve_batched(self._h, ctypes.byref(p), 1, None, None,
                                             psi.data_ptr(), infos, None, 0,
                                             _stream_handle(stream))
        if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE) or (
                raise_on_status and st != _ffi.PSI_OK):
            _check(st)
        out = []
        for i in range(self.n_graphs):
            d = _ffi.struct_dict(infos[i])
            d["status_name"] = _ffi.STATUS_NAMES.get(d["status"], str(d["status"]))
            out.append(d)
        return psi, out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.psi_operator_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_operator(graph, flags: int = 0, stream=None, device=None) -> Operator:
    """Operator from a synthetic graph record (host arrays)."""
    return Operator(graph.n, graph.follower, graph.leader, graph.lam, graph.mu,
                    node_offsets=graph.node_offsets, flags=flags, stream=stream, device=device)


# ---------------------------------------------------------------------- gather probe
def gather_probe(n_x: int, n_idx: int, col_segments: int = 1, seed: int = 0, reps: int = 20,
                 grid: int = 0, device=None, stream=None) -> dict:
    """psi_gather_probe on a random FP64 vector of n_x entries and n_idx
    random indices (uniform within a segment): the random-gather rate of an
    operator pass with that many users, edges and column segments."""
    dev = _device(device)
    gen = torch.Generator(device=dev).manual_seed(seed)
    x = torch.rand(n_x, dtype=torch.float64, device=dev, generator=gen)
    seg = n_x // col_segments
    idx = torch.randint(0, seg, (n_idx,), dtype=torch.int32, device=dev, generator=gen)
    if grid == 0:
        grid = 8 * 1024
    out = torch.empty(grid, dtype=torch.float64, device=dev)
    ms = ctypes.c_double()
    with torch.cuda.device(dev):
        _check(_ffi.load().psi_gather_probe(x.data_ptr(), n_x, col_segments, idx.data_ptr(), n_idx,
                                            out.data_ptr(), grid, reps, ctypes.byref(ms),
                                            _stream_handle(stream)))
    return dict(ms=ms.value, gathers_per_s=n_idx / (ms.value * 1e-3))


# ---------------------------------------------------------------------- learned warm start
def mpnn_param_count() -> int:
    return int(_ffi.load().psi_mpnn_param_count())


class Model:
    """The warm-start network (psi_model_*): FP32 parameters on the device,
    Adam state, and the forward / backward / update calls of psi.h.

    params: numpy float32 vector of mpnn_param_count() values (host copy)."""

    def __init__(self, params, device=None, stream=None):
        lib = _ffi.load()
        self._lib = lib
        self.device = _device(device)
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (mpnn_param_count(),):
            raise ValueError(f"params must have {mpnn_param_count()} values")
        nbytes = ctypes.c_size_t()
        _check(lib.psi_model_state_size(ctypes.byref(nbytes)))
        self.state = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.psi_model_create(p.ctypes.data, p.size, PSI_INPUT_HOST,
                                        self.state.data_ptr(), nbytes.value,
                                        _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._ws = {}

    def params(self) -> np.ndarray:
        out = np.empty(mpnn_param_count(), dtype=np.float32)
        _check(self._lib.psi_model_params(self._h, out.ctypes.data, PSI_INPUT_HOST,
                                          _stream_handle(None)))
        return out

    def grad(self) -> np.ndarray:
        out = np.empty(mpnn_param_count(), dtype=np.float32)
        _check(self._lib.psi_model_grad(self._h, out.ctypes.data, PSI_INPUT_HOST,
                                        _stream_handle(None)))
        return out

    def workspace(self, op: Operator, training: bool) -> torch.Tensor:
        """One device workspace, grown to the largest size asked for so far."""
        nb = ctypes.c_size_t()
        _check(self._lib.psi_mpnn_workspace_size(op.handle, int(training), ctypes.byref(nb)))
        ws = self._ws.get("buf")
        if ws is None or ws.numel() < nb.value:
            self._ws["buf"] = None
            ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            self._ws["buf"] = ws
        return ws

    def forward(self, op: Operator, want_t_hat: bool = True, want_s0: bool = True, stream=None):
        ws = self.workspace(op, False)
        t_hat = torch.empty(op.n, dtype=torch.float32, device=self.device) if want_t_hat else None
        s0 = torch.empty(op.n, dtype=torch.float64, device=self.device) if want_s0 else None
        _check(self._lib.psi_mpnn_forward(self._h, op.handle, _ptr(t_hat), _ptr(s0),
                                          ws.data_ptr(), ws.numel(), _stream_handle(stream)))
        return t_hat, s0

    def warmstart(self, op: Operator, s0_out: torch.Tensor | None = None, stream=None):
        ws = self.workspace(op, False)
        s0 = _vec_out(s0_out, op.n, self.device, torch.float64, "s0_out")
        _check(self._lib.psi_warmstart(self._h, op.handle, s0.data_ptr(), ws.data_ptr(),
                                       ws.numel(), _stream_handle(stream)))
        return s0

    def loss_backward(self, op: Operator, s_target: torch.Tensor, want_t_hat: bool = False,
                      stream=None):
        """Returns (loss, t_hat or None); the gradient stays in the model."""
        ws = self.workspace(op, True)
        s_target = _vec_in(s_target, op.n, self.device, torch.float64, "s_target")
        t_hat = torch.empty(op.n, dtype=torch.float32, device=self.device) if want_t_hat else None
        loss = ctypes.c_double()
        _check(self._lib.psi_mpnn_loss_backward(self._h, op.handle, s_target.data_ptr(),
                                                ctypes.byref(loss), _ptr(t_hat), ws.data_ptr(),
                                                ws.numel(), _stream_handle(stream)))
        return loss.value, t_hat

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8, stream=None):
        _check(self._lib.psi_mpnn_adam_step(self._h, lr, beta1, beta2, eps,
                                            _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.psi_model_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------- PageRank mode
def pagerank(n_users, follower, leader, alpha: float = 0.85, tol: float = 1e-9,
             power_method: bool = True, max_iter: int = 10000, op: Operator | None = None,
             stream=None):
    """psi_pagerank: PageRank by the Power-ψ kernels (Sec. III-D: with
    homogeneous activity λ = 1 − α, μ = α the ψ-score is the PageRank vector of
    eq. pagerank_power; users who follow nobody leak their mass).

    With ``power_method`` the iterates are those of the PageRank power method
    itself (the library starts from π_0 uniform and applies ``tol`` to
    ‖π_t − π_{t−1}‖₁); without it the solve is plain Power-ψ from s_0 = c with
    s-tolerance ``tol``.  Returns (pi, info, op); pass ``op`` (built with that
    activity) to reuse it.
    """
    n = int(n_users)
    if op is None:
        op = Operator(n, follower, leader, np.full(n, 1.0 - alpha), np.full(n, alpha),
                      stream=stream)
    p = op._params(tol, "abs_l1", max_iter, "fp64", 0)
    pi = torch.empty(op.n, dtype=torch.float64, device=op.device)
    start = torch.empty(op.n, dtype=torch.float64, device=op.device) if power_method else None
    info = _ffi.Info()
    with torch.cuda.device(op.device):
        st = op._lib.psi_pagerank(op._h, float(alpha), ctypes.byref(p), 1 if power_method else 0,
                                  _ptr(start), _ptr(pi), ctypes.byref(info),
                                  _stream_handle(stream))
    d = _ffi.struct_dict(info)
    d["status_name"] = _ffi.STATUS_NAMES.get(st, str(st))
    if st in (_ffi.PSI_EINVAL, _ffi.PSI_EDEVICE, _ffi.PSI_ENOSPACE):
        _check(st)
    return pi, d, op
