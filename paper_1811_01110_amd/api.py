"""Python binding of libtsqbx.so: argument marshalling only.

Every step of the evaluation runs in the library's HIP kernels.  torch
supplies device memory and streams for the asynchronous entry points.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import _lib as L

SLP, DLP, SPRIME, HELMHOLTZ = L.SLP, L.DLP, L.SPRIME, L.HELMHOLTZ
ACCUMULATE, NO_REORDER, PER_TARGET, P_MAX = L.ACCUMULATE, L.NO_REORDER, L.PER_TARGET, L.P_MAX
LAYER_BITS = (SLP, DLP, SPRIME)  # the order of every (slp, dlp, sprime) tuple


class TsqbxError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"tsqbx error {code}: {message}")
        self.code = code


def _lib():
    return L.load()


def _check(rc: int):
    if rc != 0:
        msg = _lib().tsqbx_last_error()
        raise TsqbxError(rc, msg.decode() if msg else "")


def _f64(a, cols=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if cols is not None and a.size:
        a = a.reshape(-1, cols)
    return a


def _ptr(a):
    """Data pointer of an array (NULL only for None; empty arrays stay non-NULL)."""
    return None if a is None else a.ctypes.data


def _stream_handle(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tensor_ptr(t, n, name):
    if t is None:
        return None
    import torch

    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr() if n else None


def _complex_ptr(t, n, name):
    if t is None:
        return None
    import torch

    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr() if n else None


def make_desc(sources, weights, normals, centers, list_offsets, list_sources, targets,
              target_center=None, target_normals=None):
    """A tsqbx_geometry_desc plus the arrays it points into (keep both alive)."""
    keep = dict(
        sources=_f64(sources, 3), weights=_f64(weights),
        normals=None if normals is None else _f64(normals, 3),
        centers=_f64(centers, 3),
        list_offsets=np.ascontiguousarray(list_offsets, dtype=np.int64),
        list_sources=np.ascontiguousarray(list_sources, dtype=np.int32),
        targets=_f64(targets, 3),
        target_center=None if target_center is None else np.ascontiguousarray(target_center, dtype=np.int32),
        target_normals=None if target_normals is None else _f64(target_normals, 3),
    )
    d = L.GeometryDesc(
        len(keep["weights"]), _ptr(keep["sources"]), _ptr(keep["weights"]), _ptr(keep["normals"]),
        len(keep["list_offsets"]) - 1, _ptr(keep["centers"]), keep["list_offsets"].ctypes.data,
        _ptr(keep["list_sources"]), keep["targets"].shape[0] if keep["targets"].size else 0,
        _ptr(keep["targets"]), _ptr(keep["target_center"]), _ptr(keep["target_normals"]))
    return d, keep


def validate_geometry(**arrays) -> None:
    """Host-only validation of a geometry description (raises TsqbxError)."""
    d, keep = make_desc(**arrays)
    _check(_lib().tsqbx_validate_geometry(ctypes.byref(d)))


def geometry_layout(flags: int = 0, **arrays) -> dict:
    """Host-only preview of the device layout of a geometry (no device):
    source_order, target_order, target_row, row_offsets and rows as numpy
    arrays, with the counts of tsqbx_layout_info."""
    d, keep = make_desc(**arrays)
    info = L.LayoutInfo()
    lib = _lib()
    _check(lib.tsqbx_geometry_layout(ctypes.byref(d), int(flags), None, None, None, None, 0,
                                     None, 0, ctypes.byref(info)))
    N, T = int(d.n_sources), int(d.n_targets)
    out = {"source_order": np.zeros(N, dtype=np.int64), "target_order": np.zeros(T, dtype=np.int64),
           "target_row": np.zeros(T, dtype=np.int64),
           "row_offsets": np.zeros(info.n_rows + 1, dtype=np.int64),
           "rows": np.zeros(info.nnz, dtype=np.int32)}
    _check(lib.tsqbx_geometry_layout(ctypes.byref(d), int(flags), _ptr(out["source_order"]),
                                     _ptr(out["target_order"]), _ptr(out["target_row"]),
                                     _ptr(out["row_offsets"]), info.n_rows + 1, _ptr(out["rows"]),
                                     info.nnz, ctypes.byref(info)))
    out.update({k: getattr(info, k) for k, _ in info._fields_})
    return out


def schedule_preview(items, group_lanes: int = 16, max_waves: int = 49152):
    """Host-only preview of a plan's static schedule (no device needed).

    items: sequence of (row_len, p, layers), row_len the list length of each
    target in device order.  Returns (units, wave_begin): units an (n, 3)
    int32 array of (item, first target, count), wave w working through
    units[wave_begin[w]:wave_begin[w + 1]]."""
    n = len(items)
    nt = np.array([len(r) for r, _, _ in items], dtype=np.int64)
    rl = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=np.int64) for r, _, _ in items])
                              if n else np.zeros(0, dtype=np.int64))
    ps = np.array([p for _, p, _ in items], dtype=np.int32)
    ls = np.array([l for _, _, l in items], dtype=np.uint32)
    cap = int(nt.sum()) + 1
    units = np.zeros((cap, 3), dtype=np.int32)
    wb = np.zeros(max_waves + 1, dtype=np.int32)
    nu = ctypes.c_int64(0)
    nw = ctypes.c_int32(0)
    _check(_lib().tsqbx_schedule_preview(n, _ptr(nt), _ptr(rl), _ptr(ps), _ptr(ls),
                                         int(group_lanes), int(max_waves), _ptr(units), cap,
                                         ctypes.byref(nu), _ptr(wb), ctypes.byref(nw)))
    return units[:nu.value].copy(), wb[:nw.value + 1].copy()


class Context:
    """A library context on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(_lib().tsqbx_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _check(_lib().tsqbx_ctx_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- geometry ---------------------------------------------------------
    def geometry_device(self, *, sources, weights, centers, list_offsets, list_sources, targets,
                        normals=None, target_center=None, target_normals=None, flags: int = 0,
                        stream=None) -> "Geometry":
        """Build a geometry from CUDA tensors (float64 [n][3] points, float64
        weights, int64 offsets, int32 lists and target centers) on the device:
        the same geometry as geometry() on the same arrays."""
        def ptr(t, n, cols, dtype, name):
            if t is None:
                return None
            import torch

            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and
                    t.is_contiguous() and t.numel() == n * cols):
                raise ValueError(f"{name} must be a contiguous CUDA tensor of {n * cols} {dtype}")
            return ctypes.c_void_p(t.data_ptr())
        import torch

        N, M, T = int(weights.numel()), int(centers.numel() // 3), int(targets.numel() // 3)
        nnz = int(list_sources.numel())
        d = L.GeometryDesc(
            N, ptr(sources, N, 3, torch.float64, "sources"), ptr(weights, N, 1, torch.float64, "weights"),
            ptr(normals, N, 3, torch.float64, "normals"), M,
            ptr(centers, M, 3, torch.float64, "centers"),
            ptr(list_offsets, M + 1, 1, torch.int64, "list_offsets"),
            ptr(list_sources, nnz, 1, torch.int32, "list_sources") if nnz else None, T,
            ptr(targets, T, 3, torch.float64, "targets"),
            ptr(target_center, T, 1, torch.int32, "target_center"),
            ptr(target_normals, T, 3, torch.float64, "target_normals"))
        h = ctypes.c_void_p()
        _check(_lib().tsqbx_geometry_create_device(self.handle, ctypes.byref(d), int(flags),
                                                   _stream_handle(stream), ctypes.byref(h)))
        return Geometry(self, handle=h)

    def geometry(self, g=None, *, flags: int = 0, **arrays) -> "Geometry":
        """Upload a workload Geometry (or keyword arrays) to the device."""
        if g is not None:
            arrays = dict(sources=g.sources, weights=g.weights, normals=g.normals,
                          centers=g.centers, list_offsets=g.list_offsets,
                          list_sources=g.list_sources, targets=g.targets,
                          target_center=g.target_center,
                          target_normals=getattr(g, "target_normals", None))
        return Geometry(self, flags=flags, **arrays)

    # -- evaluation ---------------------------------------------------------
    def eval(self, geom: "Geometry", sigma, p: int, layers: int, out_slp=None, out_dlp=None,
             out_sprime=None, flags: int = 0):
        """Synchronous evaluation with host arrays; returns (slp, dlp, sprime),
        None for a layer not requested."""
        sig = _f64(sigma)
        if sig.size != geom.n_sources:
            raise ValueError(f"sigma has {sig.size} entries, expected {geom.n_sources}")
        T = geom.n_targets
        outs = [out_slp, out_dlp, out_sprime]
        for k, bit in enumerate(LAYER_BITS):
            if not layers & bit:
                outs[k] = None
                continue
            if outs[k] is None:
                outs[k] = np.zeros(T)
            o = outs[k]
            if o.dtype != np.float64 or not o.flags.c_contiguous or o.size != T:
                raise ValueError("outputs must be contiguous float64 arrays of n_targets entries")
        _check(_lib().tsqbx_eval(self.handle, geom.handle, int(p), int(layers), _ptr(sig),
                                 *[_ptr(o) for o in outs], int(flags)))
        return tuple(outs)

    def eval_async(self, geom: "Geometry", sigma, p: int, layers: int, out_slp=None,
                   out_dlp=None, out_sprime=None, flags: int = 0, stream=None):
        """Asynchronous evaluation on device tensors (torch, float64)."""
        s = _tensor_ptr(sigma, geom.n_sources, "sigma")
        ptrs = [_tensor_ptr(o, geom.n_targets, name) if layers & bit else None
                for o, bit, name in zip((out_slp, out_dlp, out_sprime), LAYER_BITS,
                                        ("out_slp", "out_dlp", "out_sprime"))]
        _check(_lib().tsqbx_eval_async(self.handle, geom.handle, int(p), int(layers), s, *ptrs,
                                       int(flags), _stream_handle(stream)))

    def eval_async_noalloc(self, geom: "Geometry", sigma, p: int, layers: int, out_slp=None,
                           out_dlp=None, out_sprime=None, flags: int = 0, stream=None):
        """eval_async staged in the library's static scratch array: the call
        allocates nothing (calls overlapping on one GPU race)."""
        s = _tensor_ptr(sigma, geom.n_sources, "sigma")
        ptrs = [_tensor_ptr(o, geom.n_targets, name) if layers & bit else None
                for o, bit, name in zip((out_slp, out_dlp, out_sprime), LAYER_BITS,
                                        ("out_slp", "out_dlp", "out_sprime"))]
        _check(_lib().tsqbx_eval_async_noalloc(self.handle, geom.handle, int(p), int(layers), s,
                                               *ptrs, int(flags), _stream_handle(stream)))

    def stage_async(self, geom: "Geometry", sigma, layers: int, stream=None):
        """Strengths q = w sigma (and q nu for the double layer) into the
        geometry's staging buffer, for eval_staged_async."""
        s = _tensor_ptr(sigma, geom.n_sources, "sigma")
        _check(_lib().tsqbx_stage_async(self.handle, geom.handle, int(layers), s,
                                        _stream_handle(stream)))

    def eval_staged_async(self, geom: "Geometry", p: int, layers: int, out_slp=None,
                          out_dlp=None, out_sprime=None, flags: int = 0, stream=None):
        """Evaluation from the strengths stage_async left in the geometry."""
        ptrs = [_tensor_ptr(o, geom.n_targets, name) if layers & bit else None
                for o, bit, name in zip((out_slp, out_dlp, out_sprime), LAYER_BITS,
                                        ("out_slp", "out_dlp", "out_sprime"))]
        _check(_lib().tsqbx_eval_staged_async(self.handle, geom.handle, int(p), int(layers),
                                              *ptrs, int(flags), _stream_handle(stream)))

    def qbxl_form_async(self, geom: "Geometry", sigma, p: int, coeffs, flags: int = 0,
                        stream=None):
        """Conventional QBX: local coefficients of every center a target uses
        into coeffs, a float64 CUDA tensor of n_centers * (p+1)^2 entries
        (compact real layout)."""
        s = _tensor_ptr(sigma, geom.n_sources, "sigma")
        c = _tensor_ptr(coeffs, geom.n_centers * (p + 1) ** 2, "coeffs")
        _check(_lib().tsqbx_qbxl_form_async(self.handle, geom.handle, int(p), s, c, int(flags),
                                            _stream_handle(stream)))

    def qbxl_eval_async(self, geom: "Geometry", coeffs, p: int, out, flags: int = 0,
                        stream=None):
        """Conventional QBX: the local expansions in coeffs evaluated at the targets."""
        c = _tensor_ptr(coeffs, geom.n_centers * (p + 1) ** 2, "coeffs")
        o = _tensor_ptr(out, geom.n_targets, "out")
        _check(_lib().tsqbx_qbxl_eval_async(self.handle, geom.handle, int(p), c, o, int(flags),
                                            _stream_handle(stream)))

    def eval_conventional_async(self, geom: "Geometry", sigma, p: int, out, flags: int = 0,
                                stream=None):
        """Conventional QBX single layer, formation and evaluation in one launch."""
        s = _tensor_ptr(sigma, geom.n_sources, "sigma")
        o = _tensor_ptr(out, geom.n_targets, "out")
        _check(_lib().tsqbx_eval_conventional_async(self.handle, geom.handle, int(p), s, o,
                                                    int(flags), _stream_handle(stream)))

    def eval_helmholtz(self, geom: "Geometry", sigma, p: int, layers: int, k: float,
                       out_slp=None, out_dlp=None, out_sprime=None, flags: int = 0):
        """Helmholtz evaluation with host arrays: sigma complex (N,); returns
        complex (slp, dlp, sprime), None for a layer not requested."""
        sig = np.ascontiguousarray(sigma, dtype=np.complex128)
        if sig.size != geom.n_sources:
            raise ValueError(f"sigma has {sig.size} entries, expected {geom.n_sources}")
        T = geom.n_targets
        outs = [out_slp, out_dlp, out_sprime]
        for i, bit in enumerate(LAYER_BITS):
            if not layers & bit:
                outs[i] = None
                continue
            if outs[i] is None:
                outs[i] = np.zeros(T, dtype=np.complex128)
            o = outs[i]
            if o.dtype != np.complex128 or not o.flags.c_contiguous or o.size != T:
                raise ValueError("outputs must be contiguous complex128 arrays of n_targets entries")
        _check(_lib().tsqbx_eval_helmholtz(self.handle, geom.handle, int(p), int(layers), float(k),
                                           _ptr(sig), *[_ptr(o) for o in outs], int(flags)))
        return tuple(outs)

    def eval_helmholtz_async(self, geom: "Geometry", sigma, p: int, layers: int, k: float,
                             out_slp=None, out_dlp=None, out_sprime=None, flags: int = 0,
                             stream=None):
        """Helmholtz evaluation on device tensors (torch complex128)."""
        s = _complex_ptr(sigma, geom.n_sources, "sigma")
        outs = [_complex_ptr(o, geom.n_targets, name) if layers & bit else None
                for o, bit, name in zip((out_slp, out_dlp, out_sprime), LAYER_BITS,
                                        ("out_slp", "out_dlp", "out_sprime"))]
        _check(_lib().tsqbx_eval_helmholtz_async(self.handle, geom.handle, int(p), int(layers),
                                                 float(k), s, *outs, int(flags),
                                                 _stream_handle(stream)))

    def ball_lists(self, sources, centers, radius: float, capacity=None, stream=None):
        """Near-field lists on the device: for each center, the sources in the
        closed ball of `radius`, ascending (CSR).  sources / centers: (N, 3) /
        (M, 3) float64, numpy (copied to the device) or CUDA tensors.  Returns
        torch tensors (offsets int64 [M+1], indices int32 [nnz]) on the device."""
        import torch

        src, ctr = self._points(sources), self._points(centers)
        M = ctr.shape[0]
        offsets = torch.empty(M + 1, device=src.device, dtype=torch.int64)
        cap = int(capacity) if capacity is not None else 0
        for attempt in range(2):
            idx = torch.empty(max(cap, 1), device=src.device, dtype=torch.int32)
            nnz = ctypes.c_int64()
            rc = _lib().tsqbx_ball_lists(self.handle, src.shape[0], src.data_ptr() if src.numel() else None,
                                         M, ctr.data_ptr() if ctr.numel() else None, float(radius),
                                         offsets.data_ptr(), idx.data_ptr(), cap, ctypes.byref(nnz),
                                         _stream_handle(stream))
            if rc == L.E_RANGE and nnz.value > cap and attempt == 0:
                cap = nnz.value  # first call sized the lists
                continue
            _check(rc)
            return offsets, idx[:nnz.value]
        raise TsqbxError(L.E_RANGE, "lists did not fit after resizing")

    def knn_lists(self, sources, centers, counts, stream=None):
        """Near-field lists on the device: for each center c, the counts[c]
        nearest sources (ties to the smaller index), ascending (CSR).  sources /
        centers as for ball_lists; counts (M,) integers, numpy or a CUDA
        tensor.  Returns torch tensors (offsets int64 [M+1], indices int32)."""
        import torch

        src, ctr = self._points(sources), self._points(centers)
        M = ctr.shape[0]
        cnt = counts if isinstance(counts, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(counts, dtype=np.int32))
        cnt = cnt.to(device=src.device, dtype=torch.int32).contiguous()
        if cnt.numel() != M:
            raise ValueError(f"counts has {cnt.numel()} entries, expected {M}")
        cap = int(cnt.to(torch.int64).sum().item()) if M else 0
        offsets = torch.empty(M + 1, device=src.device, dtype=torch.int64)
        idx = torch.empty(max(cap, 1), device=src.device, dtype=torch.int32)
        nnz = ctypes.c_int64()
        _check(_lib().tsqbx_knn_lists(self.handle, src.shape[0], src.data_ptr() if src.numel() else None,
                                      M, ctr.data_ptr() if M else None, cnt.data_ptr() if M else None,
                                      offsets.data_ptr(), idx.data_ptr(), max(cap, 0),
                                      ctypes.byref(nnz), _stream_handle(stream)))
        return offsets, idx[:nnz.value]

    def _points(self, a):
        """(n, 3) float64 points on this context's device (copied if needed)."""
        import torch

        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        t = t.to(device=f"cuda:{self.device}", dtype=torch.float64).contiguous()
        return t.reshape(-1, 3) if t.numel() else t.reshape(0, 3)

    # -- tuning -------------------------------------------------------------
    def get_tuning(self, p: int, layers: int, mean_list: int) -> dict:
        t = L.Tuning()
        _check(_lib().tsqbx_get_tuning(self.handle, int(p), int(layers), int(mean_list),
                                       ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, p: int, layers: int, mean_list: int, **tuning) -> None:
        cur = self.get_tuning(p, layers, mean_list)
        cur.update(tuning)
        t = L.Tuning(**cur)
        _check(_lib().tsqbx_set_tuning(self.handle, int(p), int(layers), int(mean_list),
                                       ctypes.byref(t)))

    def autotune(self, geom: "Geometry", p: int, layers: int):
        t = L.Tuning()
        ms = ctypes.c_double()
        _check(_lib().tsqbx_autotune(self.handle, geom.handle, int(p), int(layers),
                                     ctypes.byref(t), ctypes.byref(ms)))
        return t.as_dict(), ms.value

    def tuning_save(self, path: str) -> None:
        _check(_lib().tsqbx_tuning_save(self.handle, os.fsencode(path)))

    def tuning_load(self, path: str) -> int:
        n = ctypes.c_int()
        _check(_lib().tsqbx_tuning_load(self.handle, os.fsencode(path), ctypes.byref(n)))
        return n.value

    # -- batched and served -------------------------------------------------
    def plan(self, items: Sequence[dict], flags: int = 0) -> "Plan":
        return Plan(self, items, flags)

    def plan_helmholtz(self, items: Sequence[dict], flags: int = 0) -> "Plan":
        """A Helmholtz plan: items with geom, p, layers, k, sigma and the
        outputs as complex128 CUDA tensors."""
        return Plan(self, items, flags, helmholtz=True)

    def server(self, hbm_budget: int, max_slots: int) -> "Server":
        return Server(self, hbm_budget, max_slots)


class Geometry:
    """A device-resident geometry (sources, weights, normals, centers, lists, targets)."""

    def __init__(self, ctx: Context, *, flags: int = 0, handle=None, **arrays):
        if handle is None:
            d, keep = make_desc(**arrays)
            h = ctypes.c_void_p()
            _check(_lib().tsqbx_geometry_create(ctx.handle, ctypes.byref(d), int(flags),
                                                ctypes.byref(h)))
        else:
            h = handle
        self.handle = h
        self.ctx = ctx
        info = L.GeometryInfo()
        _check(_lib().tsqbx_geometry_get_info(h, ctypes.byref(info)))
        self.n_sources = info.n_sources
        self.n_targets = info.n_targets
        self.n_centers = info.n_centers
        self.nnz = info.nnz
        self.pairs = info.pairs
        self.max_list = info.max_list
        self.device_bytes = info.device_bytes
        self.has_normals = bool(info.has_normals)
        self.has_target_normals = bool(info.has_target_normals)

    def close(self):
        if self.handle:
            _check(_lib().tsqbx_geometry_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.ctx.handle:
                self.close()
        except Exception:
            pass

    def read_layout(self) -> dict:
        """The geometry's device layout read back to the host, in the form of
        geometry_layout()."""
        info = L.LayoutInfo()
        lib = _lib()
        _check(lib.tsqbx_geometry_read_layout(self.handle, None, None, None, None, 0, None, 0,
                                              ctypes.byref(info)))
        out = {"source_order": np.zeros(self.n_sources, dtype=np.int64),
               "target_order": np.zeros(self.n_targets, dtype=np.int64),
               "target_row": np.zeros(self.n_targets, dtype=np.int64),
               "row_offsets": np.zeros(info.n_rows + 1, dtype=np.int64),
               "rows": np.zeros(info.nnz, dtype=np.int32)}
        _check(lib.tsqbx_geometry_read_layout(self.handle, _ptr(out["source_order"]),
                                              _ptr(out["target_order"]), _ptr(out["target_row"]),
                                              _ptr(out["row_offsets"]), info.n_rows + 1,
                                              _ptr(out["rows"]), info.nnz, ctypes.byref(info)))
        out.update({k: getattr(info, k) for k, _ in info._fields_})
        return out

    def pair_terms(self, p: int, layers: int) -> int:
        return self.pairs * (p + 1) * bin(layers & 7).count("1")


class Plan:
    """Many (geometry, p, layers) items in one persistent, graph-replayed launch.

    items: dicts with geom, p, layers, sigma (device tensor), out_slp, out_dlp,
    out_sprime (device tensors, needed for the requested layers).
    """

    def __init__(self, ctx: Context, items: Sequence[dict], flags: int = 0, helmholtz: bool = False):
        arr = ((L.HelmItem if helmholtz else L.Item) * len(items))()
        ptr = _complex_ptr if helmholtz else _tensor_ptr
        self._keep = list(items)
        for i, it in enumerate(items):
            g = it["geom"]
            lay = int(it["layers"])
            arr[i].geom = g.handle
            arr[i].p = int(it["p"])
            arr[i].layers = lay
            if helmholtz:
                arr[i].k = float(it["k"])
            arr[i].d_sigma = ptr(it["sigma"], g.n_sources, "sigma")
            arr[i].d_out_slp = ptr(it.get("out_slp"), g.n_targets, "out_slp") if lay & SLP else None
            arr[i].d_out_dlp = ptr(it.get("out_dlp"), g.n_targets, "out_dlp") if lay & DLP else None
            arr[i].d_out_sprime = (ptr(it.get("out_sprime"), g.n_targets, "out_sprime")
                                   if lay & SPRIME else None)
        h = ctypes.c_void_p()
        create = _lib().tsqbx_plan_create_helmholtz if helmholtz else _lib().tsqbx_plan_create
        _check(create(ctx.handle, len(items), arr, int(flags), ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx

    def execute(self, stream=None):
        _check(_lib().tsqbx_plan_execute(self.handle, _stream_handle(stream)))

    def info(self) -> dict:
        i = L.PlanInfo()
        _check(_lib().tsqbx_plan_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in i._fields_}

    def get_tuning(self) -> dict:
        t = L.PlanTuning()
        _check(_lib().tsqbx_plan_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **tuning) -> None:
        cur = self.get_tuning()
        cur.update(tuning)
        t = L.PlanTuning(**cur)
        _check(_lib().tsqbx_plan_set_tuning(self.handle, ctypes.byref(t)))

    def profile(self, reps: int = 5, stream=None) -> dict:
        """Mean per-run milliseconds of the staging and evaluation kernels."""
        t = L.PlanTiming()
        _check(_lib().tsqbx_plan_profile(self.handle, int(reps), _stream_handle(stream),
                                         ctypes.byref(t)))
        return {"stage_ms": t.stage_ms, "eval_ms": t.eval_ms, "reps": t.reps}

    def autotune(self, stream=None):
        """Time the candidate tunings, keep the fastest: (tuning, eval ms)."""
        t = L.PlanTuning()
        ms = ctypes.c_double()
        _check(_lib().tsqbx_plan_autotune(self.handle, _stream_handle(stream), ctypes.byref(t),
                                          ctypes.byref(ms)))
        return t.as_dict(), ms.value

    def close(self):
        if self.handle:
            _check(_lib().tsqbx_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.ctx.handle:
                self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over device-resident geometries."""

    def __init__(self, ctx: Context, hbm_budget: int, max_slots: int):
        h = ctypes.c_void_p()
        _check(_lib().tsqbx_server_create(ctx.handle, int(hbm_budget), int(max_slots), ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx
        self._live = {}

    @staticmethod
    def request_bytes(geom: Geometry, layers: int) -> int:
        n = ctypes.c_size_t()
        _check(_lib().tsqbx_server_request_bytes(geom.handle, int(layers), ctypes.byref(n)))
        return n.value

    @staticmethod
    def request_bytes_helmholtz(geom: Geometry, p: int, layers: int) -> int:
        n = ctypes.c_size_t()
        _check(_lib().tsqbx_server_request_bytes_helmholtz(geom.handle, int(p), int(layers),
                                                           ctypes.byref(n)))
        return n.value

    def submit(self, geom: Geometry, sigma, p: int, layers: int):
        """Queue a request; returns (ticket, out_slp, out_dlp, out_sprime): host
        arrays filled on completion (None for a layer not requested)."""
        sig = _f64(sigma)
        if sig.size != geom.n_sources:
            raise ValueError("sigma has the wrong length")
        T = geom.n_targets
        outs = tuple(np.zeros(T) if layers & bit else None for bit in LAYER_BITS)
        tk = ctypes.c_uint64()
        _check(_lib().tsqbx_server_submit(self.handle, geom.handle, int(p), int(layers), _ptr(sig),
                                          *[_ptr(o) for o in outs], ctypes.byref(tk)))
        self._live[tk.value] = outs
        return (tk.value,) + outs

    def submit_helmholtz(self, geom: Geometry, sigma, p: int, layers: int, k: float):
        """Queue a Helmholtz request (sigma complex, copied); returns (ticket,
        out_slp, out_dlp, out_sprime): complex host arrays filled on completion
        (None for a layer not requested)."""
        sig = np.ascontiguousarray(sigma, dtype=np.complex128)
        if sig.size != geom.n_sources:
            raise ValueError("sigma has the wrong length")
        T = geom.n_targets
        outs = tuple(np.zeros(T, dtype=np.complex128) if layers & bit else None for bit in LAYER_BITS)
        tk = ctypes.c_uint64()
        _check(_lib().tsqbx_server_submit_helmholtz(self.handle, geom.handle, int(p), int(layers),
                                                    float(k), _ptr(sig), *[_ptr(o) for o in outs],
                                                    ctypes.byref(tk)))
        self._live[tk.value] = outs
        return (tk.value,) + outs

    def submit_pinned(self, geom: Geometry, sigma, p: int, layers: int, out_slp=None,
                      out_dlp=None, out_sprime=None):
        """Queue a request on pinned host tensors (torch, float64), without copies.

        sigma and the outputs (allocated pinned if not given) must stay valid
        until the ticket completes.  Returns (ticket, out_slp, out_dlp, out_sprime).
        """
        return self._submit_pinned(geom, sigma, p, layers, (out_slp, out_dlp, out_sprime), None)

    def submit_helmholtz_pinned(self, geom: Geometry, sigma, p: int, layers: int, k: float,
                                out_slp=None, out_dlp=None, out_sprime=None):
        """submit_pinned for a Helmholtz request (complex128 pinned tensors)."""
        return self._submit_pinned(geom, sigma, p, layers, (out_slp, out_dlp, out_sprime), k)

    def _submit_pinned(self, geom, sigma, p, layers, outs_in, k):
        import torch

        dtype = torch.float64 if k is None else torch.complex128

        def pinned(t, n, name):
            if t is None:
                return None
            # whether the memory is pinned is checked by the library
            if t.is_cuda or t.dtype != dtype or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dtype} CPU tensor")
            if t.numel() != n:
                raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
            return t

        T = geom.n_targets
        sigma = pinned(sigma, geom.n_sources, "sigma")
        outs = []
        for o, bit, name in zip(outs_in, LAYER_BITS, ("out_slp", "out_dlp", "out_sprime")):
            if not layers & bit:
                outs.append(None)
                continue
            if o is None:
                o = torch.empty(T, dtype=dtype, pin_memory=True)
            outs.append(pinned(o, T, name))
        tk = ctypes.c_uint64()
        ptrs = [sigma.data_ptr() if sigma is not None else None] + \
            [o.data_ptr() if o is not None else None for o in outs]
        if k is None:
            _check(_lib().tsqbx_server_submit_pinned(self.handle, geom.handle, int(p), int(layers),
                                                     *ptrs, ctypes.byref(tk)))
        else:
            _check(_lib().tsqbx_server_submit_helmholtz_pinned(
                self.handle, geom.handle, int(p), int(layers), float(k), *ptrs, ctypes.byref(tk)))
        self._live[tk.value] = tuple(outs) + (sigma,)
        return (tk.value,) + tuple(outs)

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int()
        _check(_lib().tsqbx_server_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(done)))
        return bool(done.value)

    def wait(self, ticket: int, timeout_s: float = 60.0):
        _check(_lib().tsqbx_server_wait(self.handle, ctypes.c_uint64(ticket), float(timeout_s)))
        return self._live.pop(ticket, (None, None, None))[:3]

    def get_tuning(self) -> dict:
        t = L.ServerTuning()
        _check(_lib().tsqbx_server_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **tuning) -> None:
        """Only before the first submission (TSQBX_E_STATE after it)."""
        cur = self.get_tuning()
        cur.update(tuning)
        t = L.ServerTuning(**cur)
        _check(_lib().tsqbx_server_set_tuning(self.handle, ctypes.byref(t)))

    def autotune(self, requests, n_requests: int = 256, sigmas=None):
        """requests: sequence of (geometry, p, layers) cycled over by the
        bursts; sigmas: matching pinned host tensors (float64) of densities,
        or None for densities of ones.  Returns (tuning dict, best burst ms)."""
        n = len(requests)
        geoms = (ctypes.c_void_p * n)(*[g.handle for g, _, _ in requests])
        ps = np.array([p for _, p, _ in requests], dtype=np.int32)
        ls = np.array([l for _, _, l in requests], dtype=np.uint32)
        sig = None
        if sigmas is not None:
            if len(sigmas) != n:
                raise ValueError("one density per request")
            sig = (ctypes.c_void_p * n)(*[s.data_ptr() for s in sigmas])
        t = L.ServerTuning()
        ms = ctypes.c_double()
        _check(_lib().tsqbx_server_autotune(self.handle, n, ctypes.cast(geoms, ctypes.c_void_p),
                                            _ptr(ps), _ptr(ls),
                                            None if sig is None else ctypes.cast(sig, ctypes.c_void_p),
                                            int(n_requests), ctypes.byref(t), ctypes.byref(ms)))
        return t.as_dict(), ms.value

    def cancel(self, ticket: int):
        """Withdraw a request that is still queued; it then ends with
        TSQBX_E_CANCELED (wait raises it)."""
        _check(_lib().tsqbx_server_cancel(self.handle, ctypes.c_uint64(ticket)))

    def drain(self, timeout_s: float = 600.0):
        _check(_lib().tsqbx_server_drain(self.handle, float(timeout_s)))
        self._live.clear()

    def stats(self) -> dict:
        s = L.ServerStats()
        _check(_lib().tsqbx_server_get_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self.handle:
            _check(_lib().tsqbx_server_destroy(self.handle))
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            if self.ctx.handle:
                self.close()
        except Exception:
            pass
