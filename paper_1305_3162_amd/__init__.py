"""Python binding of libslp (include/slp.h): argument marshalling only.

Every arithmetic step of the single-layer-potential path runs in the HIP
library; this module converts torch device tensors and numpy host arrays into
pointers and raises SlpError on a non-zero status. If libslp.so has not been
built, importing the binding's functions raises (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "SlpError", "load_library", "expsum_sinc", "setup_geometry", "set_density",
    "set_density_from_m", "eval_single_layer", "eval_batched", "geom_get_info", "choose_cutoff", "set_graph", "set_timing", "stage_times",
    "debug_copy", "geom_destroy", "Geometry", "FP64", "FP32", "WINDOW_GAUSS", "WINDOW_KB", "STAGES",
    "geometry_device_bytes", "server_create", "server_add_geometry", "server_submit",
    "server_poll", "server_wait", "server_get_stats", "server_destroy", "Server",
    "setup_near_field", "near_radius", "near_field_info", "debug_copy_near",
    "near_pattern_host", "triangle_potential_host", "near_radius_host",
    "near_field_device_bytes", "fem_setup", "fem_info", "fem_boundary", "fem_solve_phi1", "fem_dphi1_dn",
    "scalar_potential", "fem_energy", "fem_destroy", "Fem", "fem_set_preconditioner",
    "fem_amg_info", "PRECOND_JACOBI", "PRECOND_AMG", "setup_integrated_gridding",
    "integrated_gridding_info", "amg_apply_host",
]

FP64, FP32 = 0, 1
WINDOW_GAUSS, WINDOW_KB = 0, 1
STAGES = ("spread_bins", "spread_reduce", "fft_x_fwd", "fft_y_fwd", "fft_z_mul_inv", "fft_y_inv", "fft_x_inv",
          "interp", "near")
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libslp.so")


class SlpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libslp status {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32 * 3), ("alpha", ctypes.c_int32), ("m", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("es_w", ctypes.POINTER(ctypes.c_double)),
                ("es_gamma", ctypes.POINTER(ctypes.c_double)), ("es_terms", ctypes.c_int32),
                ("window", ctypes.c_int32), ("eta2", ctypes.c_double),
                ("seg_share", ctypes.c_int32), ("reduce_cells", ctypes.c_int32)]


class GeomInfo(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_double * 3), ("scale", ctypes.c_double * 3),
                ("window_b", ctypes.c_double), ("n_nodes", ctypes.c_int64),
                ("n_tris", ctypes.c_int64), ("n_src", ctypes.c_int64),
                ("n_targets", ctypes.c_int64), ("terms_kept", ctypes.c_int32), ("lo", ctypes.c_int32 * 3),
                ("extent", ctypes.c_int32 * 3), ("tiles", ctypes.c_int32 * 3),
                ("device_bytes", ctypes.c_int64), ("seg_share", ctypes.c_int64),
                ("n_segments", ctypes.c_int64), ("reduce_cells", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("mean_s", ctypes.c_double), ("pts_per_s", ctypes.c_double),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("resident_bytes", ctypes.c_int64), ("setups", ctypes.c_int64),
                ("evictions", ctypes.c_int64), ("launches", ctypes.c_int64)]


_lib = None
_VP = ctypes.c_void_p


def load_library():
    """Load libslp.so (built in-tree by paper_1305_3162_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libslp is not built ({LIB_PATH} missing); run "
                          "`python -m paper_1305_3162_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "slp_setup_geometry": [ctypes.POINTER(_VP), _VP, ctypes.c_int64, _VP, ctypes.c_int64,
                               ctypes.POINTER(Params), _VP],
        "slp_setup_geometry_targets": [ctypes.POINTER(_VP), _VP, ctypes.c_int64, _VP,
                                       ctypes.c_int64, _VP, ctypes.c_int64,
                                       ctypes.POINTER(Params), _VP],
        "slp_set_density": [_VP, _VP, _VP],
        "slp_set_density_from_m": [_VP, _VP, _VP, _VP],
        "slp_eval_single_layer": [_VP, _VP, _VP],
        "slp_eval_single_layer_static": [_VP, _VP, _VP],
        "slp_eval_batched": [_VP, _VP, _VP, ctypes.c_int32, _VP],
        "slp_eval_batched_mode": [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP],
        "slp_geom_get_info": [_VP, ctypes.POINTER(GeomInfo)],
        "slp_set_timing": [_VP, ctypes.c_int32],
        "slp_set_graph": [_VP, ctypes.c_int32],
        "slp_choose_cutoff": [ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
        "slp_stage_times": [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                            ctypes.c_int32],
        "slp_debug_copy": [_VP, ctypes.c_int32, _VP, ctypes.c_size_t, _VP],
        "slp_expsum_sinc": [ctypes.c_double] * 4 + [_VP, _VP, ctypes.c_int32,
                                                     ctypes.POINTER(ctypes.c_int32)],
        "slp_geom_destroy": [_VP],
        "slp_geometry_device_bytes": [_VP, ctypes.c_int64, _VP, ctypes.c_int64,
                                      ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int64)],
        "slp_server_create": [ctypes.POINTER(_VP), ctypes.c_size_t, ctypes.c_int32],
        "slp_server_add_geometry": [_VP, _VP, ctypes.c_int64, _VP, ctypes.c_int64,
                                    ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int64)],
        "slp_server_submit": [_VP, ctypes.c_int64, _VP, _VP, ctypes.POINTER(ctypes.c_uint64)],
        "slp_server_poll": [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)],
        "slp_server_wait": [_VP, ctypes.c_uint64, ctypes.c_double],
        "slp_server_get_stats": [_VP, ctypes.POINTER(ServerStats), ctypes.c_int32],
        "slp_server_destroy": [_VP],
        "slp_setup_near_field": [_VP, ctypes.c_double, _VP],
        "slp_setup_near_field_stored": [_VP, ctypes.c_double, ctypes.c_int32, _VP],
        "slp_near_radius": [_VP, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
        "slp_near_field_info": [_VP, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)],
        "slp_debug_copy_near": [_VP, _VP, _VP, _VP, ctypes.c_int64],
        "slp_near_pattern_host": [_VP, ctypes.c_int64, _VP, ctypes.c_int64, _VP, ctypes.c_int64,
                                  ctypes.c_double, _VP, _VP, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_int64)],
        "slp_triangle_potential_host": [_VP, _VP, _VP, _VP, ctypes.c_int64, _VP],
        "slp_near_radius_host": [_VP, _VP, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double)],
        "slp_fem_setup": [ctypes.POINTER(_VP), _VP, ctypes.c_int64, _VP, ctypes.c_int64, _VP],
        "slp_fem_info": [_VP] + [ctypes.POINTER(ctypes.c_int64)] * 4,
        "slp_fem_boundary": [_VP, _VP, ctypes.c_int64],
        "slp_fem_solve_phi1": [_VP, _VP, _VP, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                               _VP],
        "slp_fem_dphi1_dn": [_VP, _VP, _VP, _VP],
        "slp_fem_set_preconditioner": [_VP, ctypes.c_int32, _VP],
        "slp_fem_assemble_host": [_VP, ctypes.c_int64, _VP, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  _VP, _VP, _VP, _VP],
        "slp_amg_apply_host": [ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32)],
        "slp_setup_integrated_gridding": [_VP, ctypes.c_int32, _VP],
        "slp_integrated_gridding_info": [_VP, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32)],
        "slp_fem_amg_info": [_VP, ctypes.POINTER(ctypes.c_int32), _VP, _VP, ctypes.c_int32],
        "slp_scalar_potential": [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _VP],
        "slp_fem_destroy": [_VP],
        "slp_fem_energy": [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_double), _VP],
        "slp_near_field_device_bytes": [_VP, ctypes.c_int64, _VP, ctypes.c_int64, _VP,
                                        ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64)],
        "slp_server_add_geometry_near": [_VP, _VP, ctypes.c_int64, _VP, ctypes.c_int64,
                                         ctypes.POINTER(Params), ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_int64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.slp_last_error.argtypes = []
    lib.slp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise SlpError(rc, load_library().slp_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    if stream is None:
        import torch
        return _VP(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _VP(stream)
    return _VP(stream.cuda_stream)


def _dev_f64(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements (has {t.numel()})")
    return _VP(t.data_ptr())


def expsum_sinc(h, r_lo, r_hi, tol):
    """Exponential sum for 1/r (slp_expsum_sinc): returns (omega, gamma) float64 arrays."""
    lib = load_library()
    cnt = ctypes.c_int32(0)
    lib.slp_expsum_sinc(h, r_lo, r_hi, tol, None, None, 0, ctypes.byref(cnt))
    n = cnt.value
    if n <= 0:
        _check(-1)
    w = np.empty(n)
    g = np.empty(n)
    _check(lib.slp_expsum_sinc(h, r_lo, r_hi, tol, w.ctypes.data, g.ctypes.data, n,
                               ctypes.byref(cnt)))
    return w, g


def _marshal(nodes, tris, grid, m, es_w, es_gamma, alpha, precision, eta2, window=0,
             seg_share=0, reduce_cells=0):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    if nodes.ndim != 2 or nodes.shape[1] != 3 or tris.ndim != 2 or tris.shape[1] != 3:
        raise ValueError("nodes must be [N, 3] and tris [M, 3]")
    es_w = np.ascontiguousarray(es_w, dtype=np.float64)
    es_gamma = np.ascontiguousarray(es_gamma, dtype=np.float64)
    if es_w.shape != es_gamma.shape or es_w.ndim != 1:
        raise ValueError("es_w and es_gamma must be 1-D of equal length")
    p = Params()
    p.grid[:] = [int(g) for g in grid]
    p.alpha, p.m, p.precision = int(alpha), int(m), int(precision)
    p.es_w = es_w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.es_gamma = es_gamma.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.es_terms = int(es_w.size)
    p.eta2 = float(eta2)
    p.window = int(window)
    p.seg_share = int(seg_share)
    p.reduce_cells = int(reduce_cells)
    return nodes, tris, es_w, es_gamma, p     # arrays kept alive by the caller


def setup_geometry(nodes, tris, grid, m, es_w, es_gamma, alpha=2, precision=FP64, eta2=37.0,
                   stream=None, window=WINDOW_GAUSS, targets=None, seg_share=0, reduce_cells=0):
    """slp_setup_geometry (slp_setup_geometry_targets when `targets` [P, 3] is given):
    returns an opaque handle (int). seg_share 0 = automatic gridding split;
    reduce_cells 0 = automatic block-sum form (1 or 2 cells per thread)."""
    lib = load_library()
    nodes, tris, es_w, es_gamma, p = _marshal(nodes, tris, grid, m, es_w, es_gamma, alpha,
                                              precision, eta2, window, seg_share, reduce_cells)
    h = _VP()
    if targets is None:
        _check(lib.slp_setup_geometry(ctypes.byref(h), nodes.ctypes.data, nodes.shape[0],
                                      tris.ctypes.data, tris.shape[0], ctypes.byref(p),
                                      _stream_ptr(stream)))
    else:
        targets = np.ascontiguousarray(targets, dtype=np.float64)
        if targets.ndim != 2 or targets.shape[1] != 3:
            raise ValueError("targets must be [P, 3]")
        _check(lib.slp_setup_geometry_targets(ctypes.byref(h), nodes.ctypes.data, nodes.shape[0],
                                              tris.ctypes.data, tris.shape[0],
                                              targets.ctypes.data, targets.shape[0],
                                              ctypes.byref(p), _stream_ptr(stream)))
    return h.value


def geometry_device_bytes(nodes, tris, grid, m, es_w, es_gamma, alpha=2, precision=FP64,
                          eta2=37.0, window=WINDOW_GAUSS, seg_share=0, reduce_cells=0):
    """slp_geometry_device_bytes: device bytes a context would hold (host only)."""
    lib = load_library()
    nodes, tris, es_w, es_gamma, p = _marshal(nodes, tris, grid, m, es_w, es_gamma, alpha,
                                              precision, eta2, window, seg_share, reduce_cells)
    out = ctypes.c_int64(0)
    _check(lib.slp_geometry_device_bytes(nodes.ctypes.data, nodes.shape[0], tris.ctypes.data,
                                         tris.shape[0], ctypes.byref(p), ctypes.byref(out)))
    return out.value


def server_create(device_budget_bytes, n_slots):
    h = _VP()
    _check(load_library().slp_server_create(ctypes.byref(h), int(device_budget_bytes),
                                            int(n_slots)))
    return h.value


def server_add_geometry(server, nodes, tris, grid, m, es_w, es_gamma, alpha=2, precision=FP64,
                        eta2=37.0, window=WINDOW_GAUSS, near_eps=0.0):
    """slp_server_add_geometry_near (near_eps <= 0: no near field)."""
    nodes, tris, es_w, es_gamma, p = _marshal(nodes, tris, grid, m, es_w, es_gamma, alpha,
                                              precision, eta2, window)
    gid = ctypes.c_int64(-1)
    _check(load_library().slp_server_add_geometry_near(_VP(server), nodes.ctypes.data,
                                                       nodes.shape[0], tris.ctypes.data,
                                                       tris.shape[0], ctypes.byref(p),
                                                       float(near_eps), ctypes.byref(gid)))
    return gid.value


def near_field_device_bytes(nodes, tris, eps, precision=FP64, targets=None):
    """slp_near_field_device_bytes (host only)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    out = ctypes.c_int64(0)
    if targets is None:
        tp, nt = None, 0
    else:
        targets = np.ascontiguousarray(targets, dtype=np.float64)
        tp, nt = targets.ctypes.data, targets.shape[0]
    _check(load_library().slp_near_field_device_bytes(nodes.ctypes.data, nodes.shape[0],
                                                      tris.ctypes.data, tris.shape[0], tp, nt,
                                                      float(eps), int(precision),
                                                      ctypes.byref(out)))
    return out.value


def server_submit(server, geom_id, dens, phi):
    """dens / phi: CUDA float64 tensors (kept alive by the caller until done)."""
    import torch
    for name, t in (("dens", dens), ("phi", phi)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
                or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous CUDA float64 tensor")
    tk = ctypes.c_uint64(0)
    _check(load_library().slp_server_submit(_VP(server), int(geom_id), _VP(dens.data_ptr()),
                                            _VP(phi.data_ptr()), ctypes.byref(tk)))
    return tk.value


def server_poll(server, ticket):
    done = ctypes.c_int32(0)
    _check(load_library().slp_server_poll(_VP(server), int(ticket), ctypes.byref(done)))
    return bool(done.value)


def server_wait(server, ticket, timeout_s=0.0):
    _check(load_library().slp_server_wait(_VP(server), int(ticket), float(timeout_s)))


def server_get_stats(server, reset=False):
    st = ServerStats()
    _check(load_library().slp_server_get_stats(_VP(server), ctypes.byref(st), int(bool(reset))))
    return {k: getattr(st, k) for k, _ in ServerStats._fields_}


def server_destroy(server):
    _check(load_library().slp_server_destroy(_VP(server)))


def set_density(geom, dens, stream=None):
    info = geom_get_info(geom)
    _check(load_library().slp_set_density(_VP(geom), _dev_f64(dens, info["n_src"], "dens"),
                                          _stream_ptr(stream)))


def set_density_from_m(geom, m_nodes, dphi1_dn=None, stream=None):
    """Element-constant density m.n - dphi1/dn from a nodal magnetisation, formed on
    the device (m_nodes: CUDA float64 [n_nodes, 3]; dphi1_dn: [n_tris] or None)."""
    info = geom_get_info(geom)
    mp = _dev_f64(m_nodes, 3 * info["n_nodes"], "m_nodes")
    dp = None if dphi1_dn is None else _dev_f64(dphi1_dn, info["n_tris"], "dphi1_dn")
    _check(load_library().slp_set_density_from_m(_VP(geom), mp, dp, _stream_ptr(stream)))


def eval_single_layer(geom, phi, stream=None):
    info = geom_get_info(geom)
    _check(load_library().slp_eval_single_layer(_VP(geom), _dev_f64(phi, info["n_targets"], "phi"),
                                                _stream_ptr(stream)))


# bytes of the static device workspace of eval_single_layer_static
# (SLP_STATIC_WORKSPACE_BYTES in include/slp.h)
STATIC_WORKSPACE_BYTES = 64 << 20


def eval_single_layer_static(geom, phi, stream=None):
    """slp_eval_single_layer_static: the evaluation with every work buffer in
    the library's static device workspace (allocates nothing)."""
    info = geom_get_info(geom)
    _check(load_library().slp_eval_single_layer_static(
        _VP(geom), _dev_f64(phi, info["n_targets"], "phi"), _stream_ptr(stream)))


BATCH_AUTO, BATCH_LANES, BATCH_FUSED = 0, 1, 2


def eval_batched(geoms, dens, phis, stream=None, mode=None):
    """slp_eval_batched (mode None) or slp_eval_batched_mode (BATCH_AUTO,
    BATCH_LANES or BATCH_FUSED)."""
    n = len(geoms)
    if not (len(dens) == len(phis) == n) or n < 1:
        raise ValueError("geoms, dens and phis must have the same length >= 1")
    G = (_VP * n)(*[_VP(g) for g in geoms])
    D = (_VP * n)()
    P = (_VP * n)()
    infos = {}
    for i, g in enumerate(geoms):
        info = infos.get(g)
        if info is None:
            info = infos[g] = geom_get_info(g)
        D[i] = _dev_f64(dens[i], info["n_src"], f"dens[{i}]").value
        P[i] = _dev_f64(phis[i], info["n_targets"], f"phi[{i}]").value
    if mode is None:
        _check(load_library().slp_eval_batched(G, D, P, n, _stream_ptr(stream)))
    else:
        _check(load_library().slp_eval_batched_mode(G, D, P, n, int(mode), _stream_ptr(stream)))


def geom_get_info(geom):
    gi = GeomInfo()
    _check(load_library().slp_geom_get_info(_VP(geom), ctypes.byref(gi)))
    return {"centre": list(gi.centre), "scale": list(gi.scale), "window_b": gi.window_b,
            "n_nodes": gi.n_nodes, "n_tris": gi.n_tris, "n_src": gi.n_src,
            "n_targets": gi.n_targets,
            "terms_kept": gi.terms_kept, "lo": list(gi.lo), "extent": list(gi.extent),
            "tiles": list(gi.tiles), "device_bytes": gi.device_bytes,
            "seg_share": gi.seg_share, "n_segments": gi.n_segments,
            "reduce_cells": gi.reduce_cells}


def choose_cutoff(tol, precision=FP64, window=None):
    """slp_choose_cutoff: (window, m) with the smallest m predicted to meet tol."""
    w, m = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load_library().slp_choose_cutoff(float(tol), int(precision),
                                            -1 if window is None else int(window),
                                            ctypes.byref(w), ctypes.byref(m)))
    return w.value, m.value


def set_graph(geom, enable=True):
    """Replay evaluations of this context through captured HIP graphs."""
    _check(load_library().slp_set_graph(_VP(geom), int(bool(enable))))


def set_timing(geom, every=1):
    """Record stage events on every `every`-th evaluation (0 or False: off)."""
    _check(load_library().slp_set_timing(_VP(geom), int(every)))


def stage_times(geom, reset=False):
    ms = (ctypes.c_double * len(STAGES))()
    cnt = ctypes.c_int64(0)
    _check(load_library().slp_stage_times(_VP(geom), ms, ctypes.byref(cnt), int(bool(reset))))
    return dict(zip(STAGES, list(ms))), cnt.value


def debug_copy(geom, which, dst, stream=None):
    import torch
    if not isinstance(dst, torch.Tensor) or not dst.is_cuda or not dst.is_contiguous():
        raise TypeError("dst must be a contiguous CUDA tensor")
    nbytes = dst.numel() * dst.element_size()
    _check(load_library().slp_debug_copy(_VP(geom), int(which), _VP(dst.data_ptr()), nbytes,
                                         _stream_ptr(stream)))


def setup_near_field(geom, eps, stream=None, storage=None):
    """slp_setup_near_field: near-field correction within physical distance eps
    (eps <= 0 removes it); with `storage` (FP64 / FP32) slp_setup_near_field_stored,
    the values stored in that precision."""
    if storage is None:
        _check(load_library().slp_setup_near_field(_VP(geom), float(eps), _stream_ptr(stream)))
    else:
        _check(load_library().slp_setup_near_field_stored(_VP(geom), float(eps), int(storage),
                                                          _stream_ptr(stream)))


def near_radius(geom, tol):
    """slp_near_radius: eps from which the kept exponential sum matches 1/r to tol."""
    out = ctypes.c_double(0.0)
    _check(load_library().slp_near_radius(_VP(geom), float(tol), ctypes.byref(out)))
    return out.value


def near_field_info(geom):
    eps, nnz, rmax = ctypes.c_double(0.0), ctypes.c_int64(0), ctypes.c_double(0.0)
    stored, packed = ctypes.c_int64(0), ctypes.c_int32(0)
    _check(load_library().slp_near_field_info(_VP(geom), ctypes.byref(eps), ctypes.byref(nnz),
                                              ctypes.byref(rmax), ctypes.byref(stored),
                                              ctypes.byref(packed)))
    return {"eps": eps.value, "nnz": nnz.value, "r_max": rmax.value, "stored": stored.value,
            "packed": bool(packed.value)}


def debug_copy_near(geom):
    """The near-field matrix as host arrays (rowptr int64, cols int32, vals float64)."""
    info = geom_get_info(geom)
    nnz = near_field_info(geom)["nnz"]
    rowptr = np.zeros(info["n_targets"] + 1, dtype=np.int64)
    cols = np.zeros(max(nnz, 1), dtype=np.int32)
    vals = np.zeros(max(nnz, 1), dtype=np.float64)
    _check(load_library().slp_debug_copy_near(_VP(geom), rowptr.ctypes.data, cols.ctypes.data,
                                              vals.ctypes.data, cols.size))
    return rowptr, cols[:nnz], vals[:nnz]


def near_pattern_host(nodes, tris, targets, eps):
    """slp_near_pattern_host: (rowptr, cols) of the index sets, computed on the host."""
    lib = load_library()
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    targets = np.ascontiguousarray(targets, dtype=np.float64)
    nnz = ctypes.c_int64(0)
    args = (nodes.ctypes.data, nodes.shape[0], tris.ctypes.data, tris.shape[0],
            targets.ctypes.data, targets.shape[0], float(eps))
    _check(lib.slp_near_pattern_host(*args, None, None, 0, ctypes.byref(nnz)))
    rowptr = np.zeros(targets.shape[0] + 1, dtype=np.int64)
    cols = np.zeros(max(nnz.value, 1), dtype=np.int32)
    _check(lib.slp_near_pattern_host(*args, rowptr.ctypes.data, cols.ctypes.data, cols.size,
                                     ctypes.byref(nnz)))
    return rowptr, cols[:nnz.value]


def triangle_potential_host(x, a, b, c):
    """slp_triangle_potential_host over arrays [count, 3] (broadcast first)."""
    x, a, b, c = (np.ascontiguousarray(v, dtype=np.float64)
                  for v in np.broadcast_arrays(x, a, b, c))
    shape = x.shape[:-1]
    x, a, b, c = (np.ascontiguousarray(v.reshape(-1, 3)) for v in (x, a, b, c))
    out = np.empty(x.shape[0])
    _check(load_library().slp_triangle_potential_host(x.ctypes.data, a.ctypes.data,
                                                      b.ctypes.data, c.ctypes.data,
                                                      x.shape[0], out.ctypes.data))
    return out.reshape(shape)


def near_radius_host(es_w, es_gamma, r_max, tol):
    es_w = np.ascontiguousarray(es_w, dtype=np.float64)
    es_gamma = np.ascontiguousarray(es_gamma, dtype=np.float64)
    out = ctypes.c_double(0.0)
    _check(load_library().slp_near_radius_host(es_w.ctypes.data, es_gamma.ctypes.data,
                                               es_w.size, float(r_max), float(tol),
                                               ctypes.byref(out)))
    return out.value


def fem_setup(nodes, tets, stream=None):
    """slp_fem_setup: P1 Dirichlet-problem context for a tetrahedral mesh (handle)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    if nodes.ndim != 2 or nodes.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
        raise ValueError("nodes must be [N, 3] and tets [T, 4]")
    h = _VP()
    _check(load_library().slp_fem_setup(ctypes.byref(h), nodes.ctypes.data, nodes.shape[0],
                                        tets.ctypes.data, tets.shape[0], _stream_ptr(stream)))
    return h.value


def fem_info(fem):
    v = [ctypes.c_int64(0) for _ in range(4)]
    _check(load_library().slp_fem_info(_VP(fem), *[ctypes.byref(x) for x in v]))
    return dict(zip(("n_free", "n_boundary_tris", "nnz", "device_bytes"), [x.value for x in v]))


def fem_boundary(fem):
    n = fem_info(fem)["n_boundary_tris"]
    tris = np.zeros((n, 3), dtype=np.int32)
    _check(load_library().slp_fem_boundary(_VP(fem), tris.ctypes.data, n))
    return tris


def fem_solve_phi1(fem, m_nodes, phi1, tol=1e-10, max_iter=20000, warm_start=False, stream=None):
    """slp_fem_solve_phi1 (m_nodes CUDA float64 [N, 3], phi1 CUDA float64 [N]);
    returns (iterations, relative residual)."""
    it, rr = ctypes.c_int32(0), ctypes.c_double(0.0)
    n = phi1.numel()
    _check(load_library().slp_fem_solve_phi1(_VP(fem), _dev_f64(m_nodes, 3 * n, "m_nodes"),
                                             _dev_f64(phi1, n, "phi1"), float(tol), int(max_iter),
                                             int(bool(warm_start)), ctypes.byref(it),
                                             ctypes.byref(rr), _stream_ptr(stream)))
    return it.value, rr.value


def setup_integrated_gridding(geom, order=8, stream=None):
    """slp_setup_integrated_gridding: grid the window integrated over each
    triangle (order Gauss points per direction; 0 = point gridding)."""
    _check(load_library().slp_setup_integrated_gridding(_VP(geom), int(order), _stream_ptr(stream)))


def integrated_gridding_info(geom):
    o, n, st, pk = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
    _check(load_library().slp_integrated_gridding_info(_VP(geom), ctypes.byref(o), ctypes.byref(n),
                                                       ctypes.byref(st), ctypes.byref(pk)))
    return {"order": o.value, "nnz": n.value, "stored": st.value, "packed": bool(pk.value)}


def fem_assemble_host(nodes, tets):
    """slp_fem_assemble_host: (rowptr, cols, vals, free_nodes) of the free-node
    stiffness matrix, assembled on the host."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    lib = load_library()
    nf, nnz = ctypes.c_int64(0), ctypes.c_int64(0)
    args = (nodes.ctypes.data, nodes.shape[0], tets.ctypes.data, tets.shape[0])
    _check(lib.slp_fem_assemble_host(*args, ctypes.byref(nf), ctypes.byref(nnz), None, None, None,
                                     None))
    rp = np.empty(nf.value + 1, dtype=np.int64)
    ci = np.empty(nnz.value, dtype=np.int32)
    v = np.empty(nnz.value, dtype=np.float64)
    fn = np.empty(nf.value, dtype=np.int32)
    _check(lib.slp_fem_assemble_host(*args, ctypes.byref(nf), ctypes.byref(nnz), rp.ctypes.data,
                                     ci.ctypes.data, v.ctypes.data, fn.ctypes.data))
    return rp, ci, v, fn


def amg_apply_host(rowptr, cols, vals, r):
    """slp_amg_apply_host: z = B r for one multigrid cycle built from the CSR
    matrix (host arrays); returns (z, number of operators in the hierarchy)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = rowptr.size - 1
    if r.size != n:
        raise ValueError("r must have one value per row")
    z = np.zeros(n)
    nl = ctypes.c_int32(0)
    _check(load_library().slp_amg_apply_host(n, rowptr.ctypes.data, cols.ctypes.data, vals.ctypes.data,
                                             r.ctypes.data, z.ctypes.data, ctypes.byref(nl)))
    return z, nl.value


PRECOND_JACOBI, PRECOND_AMG = 0, 1


def fem_set_preconditioner(fem, kind, stream=None):
    """slp_fem_set_preconditioner: PRECOND_JACOBI or PRECOND_AMG (or "jacobi" / "amg")."""
    kind = {"jacobi": PRECOND_JACOBI, "amg": PRECOND_AMG}.get(kind, kind)
    _check(load_library().slp_fem_set_preconditioner(_VP(fem), int(kind), _stream_ptr(stream)))


def fem_amg_info(fem):
    """slp_fem_amg_info: [(rows, stored entries)] of the hierarchy, finest first."""
    nl = ctypes.c_int32(0)
    _check(load_library().slp_fem_amg_info(_VP(fem), ctypes.byref(nl), None, None, 0))
    rows = np.zeros(nl.value, dtype=np.int64)
    nnz = np.zeros(nl.value, dtype=np.int64)
    _check(load_library().slp_fem_amg_info(_VP(fem), ctypes.byref(nl), rows.ctypes.data,
                                           nnz.ctypes.data, nl.value))
    return list(zip(rows.tolist(), nnz.tolist()))


def fem_dphi1_dn(fem, phi1, dn, stream=None):
    n = fem_info(fem)["n_boundary_tris"]
    _check(load_library().slp_fem_dphi1_dn(_VP(fem), _dev_f64(phi1, phi1.numel(), "phi1"),
                                           _dev_f64(dn, n, "dphi1_dn"), _stream_ptr(stream)))


def scalar_potential(fem, geom, m_nodes, phi, tol=1e-10, max_iter=20000, warm_start=False,
                     stream=None):
    """slp_scalar_potential: phi = phi_1 + phi_2 at every node; returns the CG iterations."""
    it = ctypes.c_int32(0)
    n = phi.numel()
    _check(load_library().slp_scalar_potential(_VP(fem), _VP(geom),
                                               _dev_f64(m_nodes, 3 * n, "m_nodes"),
                                               _dev_f64(phi, n, "phi"), float(tol), int(max_iter),
                                               int(bool(warm_start)), ctypes.byref(it),
                                               _stream_ptr(stream)))
    return it.value


def fem_energy(fem, m_nodes, phi, stream=None):
    """slp_fem_energy: (1/2) int m . grad phi over the mesh."""
    e = ctypes.c_double(0.0)
    n = phi.numel()
    _check(load_library().slp_fem_energy(_VP(fem), _dev_f64(m_nodes, 3 * n, "m_nodes"),
                                         _dev_f64(phi, n, "phi"), ctypes.byref(e),
                                         _stream_ptr(stream)))
    return e.value


def fem_destroy(fem):
    _check(load_library().slp_fem_destroy(_VP(fem)))


def geom_destroy(geom):
    _check(load_library().slp_geom_destroy(_VP(geom)))


class Geometry:
    """Owning wrapper around one slp_geom context."""

    def __init__(self, nodes, tris, grid, m, es_w, es_gamma, alpha=2, precision=FP64,
                 eta2=37.0, stream=None, window=WINDOW_GAUSS, targets=None, seg_share=0,
                 reduce_cells=0):
        self.handle = setup_geometry(nodes, tris, grid, m, es_w, es_gamma, alpha, precision,
                                     eta2, stream, window, targets, seg_share, reduce_cells)
        self.info = geom_get_info(self.handle)
        self.precision = precision

    def set_density(self, dens, stream=None):
        set_density(self.handle, dens, stream)

    def set_density_from_m(self, m_nodes, dphi1_dn=None, stream=None):
        set_density_from_m(self.handle, m_nodes, dphi1_dn, stream)

    def eval(self, phi, stream=None):
        eval_single_layer(self.handle, phi, stream)

    def setup_near_field(self, eps, stream=None, storage=None):
        setup_near_field(self.handle, eps, stream, storage)
        self.info = geom_get_info(self.handle)

    def near_radius(self, tol):
        return near_radius(self.handle, tol)

    def near_field_info(self):
        return near_field_info(self.handle)

    def setup_integrated_gridding(self, order=8, stream=None):
        setup_integrated_gridding(self.handle, order, stream)

    def integrated_gridding_info(self):
        return integrated_gridding_info(self.handle)

    def solve(self, dens, stream=None):
        import torch
        phi = torch.empty(self.info["n_targets"], dtype=torch.float64, device=dens.device)
        self.set_density(dens, stream)
        self.eval(phi, stream)
        return phi

    def close(self):
        if self.handle:
            geom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fem:
    """Owning wrapper around one slp_fem context."""

    def __init__(self, nodes, tets, stream=None, precond="jacobi"):
        self.handle = fem_setup(nodes, tets, stream)
        if precond != "jacobi":
            fem_set_preconditioner(self.handle, precond, stream)
        self.info = fem_info(self.handle)
        self.boundary = fem_boundary(self.handle)

    def solve_phi1(self, m_nodes, phi1, tol=1e-10, max_iter=20000, warm_start=False, stream=None):
        return fem_solve_phi1(self.handle, m_nodes, phi1, tol, max_iter, warm_start, stream)

    def dphi1_dn(self, phi1, dn, stream=None):
        fem_dphi1_dn(self.handle, phi1, dn, stream)

    def energy(self, m_nodes, phi, stream=None):
        return fem_energy(self.handle, m_nodes, phi, stream)

    def close(self):
        if self.handle:
            fem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Owning wrapper around one slp_server (queued / served evaluation)."""

    def __init__(self, device_budget_bytes, n_slots=4):
        self.handle = server_create(device_budget_bytes, n_slots)

    def add_geometry(self, nodes, tris, grid, m, es_w, es_gamma, alpha=2, precision=FP64,
                     eta2=37.0, window=WINDOW_GAUSS, near_eps=0.0):
        return server_add_geometry(self.handle, nodes, tris, grid, m, es_w, es_gamma, alpha,
                                   precision, eta2, window, near_eps)

    def submit(self, geom_id, dens, phi):
        return server_submit(self.handle, geom_id, dens, phi)

    def poll(self, ticket):
        return server_poll(self.handle, ticket)

    def wait(self, ticket, timeout_s=0.0):
        server_wait(self.handle, ticket, timeout_s)

    def stats(self, reset=False):
        return server_get_stats(self.handle, reset)

    def close(self):
        if self.handle:
            server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
