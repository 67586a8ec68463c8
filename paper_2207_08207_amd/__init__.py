"""Python binding of liblst (include/lst.h): the MI355X Line Segment Tracking chain.

Argument marshalling only: every step of the chain runs in the library's HIP
kernels.  PyTorch provides device memory (input tensors, the per-event
workspace as a uint8 tensor, i.e. torch's caching allocator) and streams.
The functions named ``lst_*`` mirror the C ABI one to one; ``Geometry``,
``upload_event`` and ``run_event`` are thin conveniences over them.

The library must have been built (``paper_2207_08207_amd.build.build()``);
importing the binding on a machine without it raises ImportError, and there
is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblst.so")

LST_OK, LST_E_INVALID, LST_E_NOMEM, LST_E_CAPACITY, LST_E_DEVICE, LST_E_STATE = 0, -1, -2, -3, -4, -5
STAGES = ["MD", "LS", "T3", "T5", "pLS", "pT3", "pT5", "TC"]
TUPLE_W = [2, 4, 6, 10, 1, 7, 11]
ATTR_W = [0, 2, 4, 8, 5, 3, 3]
EXPORTED = ["lst_load_geometry", "lst_release_geometry", "lst_default_capacity", "lst_workspace_bytes",
            "lst_build_event", "lst_enqueue_event", "lst_event_query", "lst_event_wait",
            "lst_get_track_candidates", "lst_get_stage_objects", "lst_get_stage_counts",
            "lst_get_module_constants", "lst_release_event", "lst_last_error", "lst_kernel_site_count",
            "lst_kernel_site_name", "lst_set_timed_site", "lst_get_site_time", "lst_batch_workspace_bytes",
            "lst_enqueue_batch", "lst_plan_workspace_bytes", "lst_plan_create", "lst_plan_run", "lst_plan_release",
            "lst_server_create", "lst_server_now", "lst_server_submit", "lst_server_poll", "lst_server_pending",
            "lst_server_destroy", "lst_get_launch_config", "lst_set_launch_config", "lst_autotune",
            "lst_set_track_extensions", "lst_get_extended_track_candidates", "lst_set_impact_bound",
            "lst_set_stub_precision", "lst_set_t5_cuts", "lst_get_t5_cuts",
            "lst_get_default_t5_cuts", "lst_build_event_static", "lst_static_workspace_bytes",
            "lst_server_submit_with_capacity", "lst_server_reruns", "lst_tile_count", "lst_tile_name",
            "lst_tile_range", "lst_get_tile_config", "lst_set_tile_config", "lst_autotune_tiles",
            "lst_probe_valu"]


class LSTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"liblst status {status}: {msg}")
        self.status = status


class lst_geometry_desc(ctypes.Structure):
    _fields_ = [("n_modules", ctypes.c_int32),
                ("subdet", ctypes.c_void_p), ("layer", ctypes.c_void_p), ("side", ctypes.c_void_p),
                ("type", ctypes.c_void_p), ("pos_lo", ctypes.c_void_p), ("pos_up", ctypes.c_void_p),
                ("lmin", ctypes.c_void_p), ("lmax", ctypes.c_void_p), ("n_edges", ctypes.c_int32),
                ("map_offsets", ctypes.c_void_p), ("map_targets", ctypes.c_void_p)]


class lst_event_desc(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_int32), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("module", ctypes.c_void_p), ("sensor", ctypes.c_void_p),
                ("n_seeds", ctypes.c_int32), ("px", ctypes.c_void_p), ("py", ctypes.c_void_p),
                ("pz", ctypes.c_void_p), ("q", ctypes.c_void_p), ("hits4", ctypes.c_void_p)]


class lst_capacity(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("md", "ls", "t3", "t5", "pt3", "pt5")]


class lst_server_config(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class lst_server_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("event", ctypes.c_void_p), ("arrival_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double), ("status", ctypes.c_int32)]


_lib = None


def load_library(path=LIB_PATH):
    """dlopen liblst.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"liblst.so not built ({path}); run paper_2207_08207_amd.build.build()")
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library then shares)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "lst_load_geometry": [P(lst_geometry_desc), P(vp)],
        "lst_release_geometry": [vp],
        "lst_default_capacity": [i32, i32, P(lst_capacity)],
        "lst_workspace_bytes": [vp, i32, i32, P(lst_capacity), P(sz)],
        "lst_build_event": [vp, P(lst_event_desc), P(lst_capacity), vp, sz, vp, P(vp)],
        "lst_enqueue_event": [vp, P(lst_event_desc), P(lst_capacity), vp, sz, vp, P(vp)],
        "lst_event_query": [vp, P(i32)],
        "lst_event_wait": [vp],
        "lst_get_track_candidates": [vp, P(i32), P(i32), vp, vp, vp],
        "lst_set_track_extensions": [vp, i32],
        "lst_set_impact_bound": [vp, ctypes.c_double],
        "lst_set_stub_precision": [vp, i32],
        "lst_set_t5_cuts": [vp, vp, vp],
        "lst_get_t5_cuts": [vp, vp, vp],
        "lst_get_default_t5_cuts": [vp, vp],
        "lst_build_event_static": [vp, P(lst_event_desc), P(lst_capacity), vp, i32, i32, vp, vp, vp, vp],
        "lst_static_workspace_bytes": [P(sz)],
        "lst_get_extended_track_candidates": [vp, P(i32), P(i32), vp, vp, vp, vp, vp, vp],
        "lst_get_stage_objects": [vp, i32, P(i32), vp, vp, vp],
        "lst_get_stage_counts": [vp, vp, vp],
        "lst_get_module_constants": [vp, vp],
        "lst_release_event": [vp],
        "lst_set_timed_site": [i32],
        "lst_get_site_time": [vp, P(ctypes.c_float)],
        "lst_batch_workspace_bytes": [vp, i32, vp, vp, vp, P(sz)],
        "lst_enqueue_batch": [vp, i32, vp, vp, vp, sz, vp, vp],
        "lst_plan_workspace_bytes": [vp, i32, i32, i32, P(lst_capacity), P(sz)],
        "lst_plan_create": [vp, i32, i32, i32, P(lst_capacity), vp, sz, vp, P(vp)],
        "lst_plan_run": [vp, i32, vp, vp, vp],
        "lst_plan_release": [vp],
        "lst_server_create": [vp, P(lst_server_config), vp, sz, P(vp)],
        "lst_server_now": [vp, P(ctypes.c_double)],
        "lst_server_submit": [vp, P(lst_event_desc), ctypes.c_int64, ctypes.c_double],
        "lst_server_submit_with_capacity": [vp, P(lst_event_desc), P(lst_capacity), ctypes.c_int64,
                                            ctypes.c_double],
        "lst_server_reruns": [vp, P(ctypes.c_int64)],
        "lst_server_poll": [vp, vp, i32, P(i32)],
        "lst_server_pending": [vp, P(i32), P(i32)],
        "lst_server_destroy": [vp],
        "lst_get_launch_config": [vp, i32, vp],
        "lst_set_launch_config": [vp, i32, vp],
        "lst_autotune": [vp, i32, vp, vp, vp, sz, vp, i32, vp],
        "lst_autotune_tiles": [vp, i32, vp, vp, vp, sz, vp, i32, vp],
        "lst_probe_valu": [i32, i32, vp, vp],
        "lst_tile_range": [i32, P(i32), P(i32)],
        "lst_get_tile_config": [vp, i32, vp],
        "lst_set_tile_config": [vp, i32, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.lst_last_error.argtypes = []
    lib.lst_last_error.restype = ctypes.c_char_p
    lib.lst_kernel_site_count.argtypes = []
    lib.lst_kernel_site_count.restype = ctypes.c_int32
    lib.lst_kernel_site_name.argtypes = [i32]
    lib.lst_kernel_site_name.restype = ctypes.c_char_p
    lib.lst_tile_count.argtypes = []
    lib.lst_tile_count.restype = ctypes.c_int32
    lib.lst_tile_name.argtypes = [i32]
    lib.lst_tile_name.restype = ctypes.c_char_p
    _lib = lib
    return lib


def lst_last_error():
    return load_library().lst_last_error().decode(errors="replace")


def _check(status):
    if status != LST_OK:
        raise LSTError(status, lst_last_error())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


# ------------------------------------------------------------- C ABI mirror
def lst_load_geometry(subdet, layer, side, type, pos_lo, pos_up, lmin, lmax, map_offsets, map_targets):
    """Host arrays in, opaque geometry handle (int) out."""
    arrs = [np.ascontiguousarray(a, np.int32) for a in (subdet, layer, side, type)]
    arrs += [np.ascontiguousarray(a, np.float32) for a in (pos_lo, pos_up, lmin, lmax)]
    off = np.ascontiguousarray(map_offsets, np.int32)
    tgt = np.ascontiguousarray(map_targets, np.int32)
    d = lst_geometry_desc(int(arrs[0].size), *[_ptr(a) for a in arrs], int(tgt.size), _ptr(off), _ptr(tgt))
    h = ctypes.c_void_p()
    _check(load_library().lst_load_geometry(ctypes.byref(d), ctypes.byref(h)))
    return h.value


def lst_release_geometry(geom):
    _check(load_library().lst_release_geometry(geom))


def lst_default_capacity(n_hits, n_seeds):
    c = lst_capacity()
    _check(load_library().lst_default_capacity(int(n_hits), int(n_seeds), ctypes.byref(c)))
    return c


def lst_workspace_bytes(geom, n_hits, n_seeds, cap=None):
    b = ctypes.c_size_t()
    _check(load_library().lst_workspace_bytes(geom, int(n_hits), int(n_seeds),
                                              ctypes.byref(cap) if cap is not None else None, ctypes.byref(b)))
    return int(b.value)


def _event_desc(t):
    return lst_event_desc(int(t["x"].numel()), _ptr(t["x"]), _ptr(t["y"]), _ptr(t["z"]), _ptr(t["module"]),
                          _ptr(t["sensor"]), int(t["px"].numel()), _ptr(t["px"]), _ptr(t["py"]), _ptr(t["pz"]),
                          _ptr(t["q"]), _ptr(t["hits4"]))


def lst_build_event(geom, dev_event, workspace, cap=None, stream=None):
    """Runs the chain (synchronously) on device tensors; returns (status, event handle)."""
    d = _event_desc(dev_event)
    h = ctypes.c_void_p()
    st = load_library().lst_build_event(geom, ctypes.byref(d), ctypes.byref(cap) if cap is not None else None,
                                        _ptr(workspace), int(workspace.numel()), stream, ctypes.byref(h))
    return st, h.value


def lst_static_workspace_bytes():
    n = ctypes.c_size_t()
    _check(load_library().lst_static_workspace_bytes(ctypes.byref(n)))
    return int(n.value)


def lst_build_event_static(geom, dev_event, type_out, offsets_out, hits_out, counts_out, cap=None, stream=None):
    """Allocation-free build: the chain runs in the library's static workspace; the track candidates
    go to the given device int32 tensors (counts_out[0..2] = candidates, hits, status).  Returns at
    once; synchronize the stream before reading the outputs."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    if offsets_out.numel() < type_out.numel() + 1:
        raise ValueError("offsets_out needs one entry more than type_out")
    d = _event_desc(dev_event)
    c = None if cap is None else ctypes.byref(cap)
    _check(load_library().lst_build_event_static(
        geom, ctypes.byref(d), c, ctypes.c_void_p(stream), int(type_out.numel()), int(hits_out.numel()),
        ctypes.c_void_p(type_out.data_ptr()), ctypes.c_void_p(offsets_out.data_ptr()),
        ctypes.c_void_p(hits_out.data_ptr()), ctypes.c_void_p(counts_out.data_ptr())))


def lst_enqueue_event(geom, dev_event, workspace, cap=None, stream=None):
    d = _event_desc(dev_event)
    h = ctypes.c_void_p()
    st = load_library().lst_enqueue_event(geom, ctypes.byref(d), ctypes.byref(cap) if cap is not None else None,
                                          _ptr(workspace), int(workspace.numel()), stream, ctypes.byref(h))
    return st, h.value


def lst_event_query(ev):
    done = ctypes.c_int32()
    _check(load_library().lst_event_query(ev, ctypes.byref(done)))
    return bool(done.value)


def lst_event_wait(ev):
    return load_library().lst_event_wait(ev)


def lst_get_track_candidates(ev):
    lib = load_library()
    n, nh = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.lst_get_track_candidates(ev, ctypes.byref(n), ctypes.byref(nh), None, None, None))
    ty = np.zeros(n.value, np.int32)
    off = np.zeros(n.value + 1, np.int32)
    hits = np.zeros(nh.value, np.int32)
    _check(lib.lst_get_track_candidates(ev, ctypes.byref(n), ctypes.byref(nh), _ptr(ty), _ptr(off), _ptr(hits)))
    return ty, off, hits


def lst_set_stub_precision(geom, bits):
    _check(load_library().lst_set_stub_precision(geom, int(bits)))


def lst_set_impact_bound(geom, d0_max):
    _check(load_library().lst_set_impact_bound(geom, float(d0_max)))


def lst_set_t5_cuts(geom, xy=None, rz=None):
    """Quintuplet chi2 cuts of the 1024 categories (None: that half keeps the calibrated table)."""
    ax = None if xy is None else np.ascontiguousarray(np.broadcast_to(xy, (1024,)), np.float32)
    ar = None if rz is None else np.ascontiguousarray(np.broadcast_to(rz, (1024,)), np.float32)
    _check(load_library().lst_set_t5_cuts(geom, None if ax is None else _ptr(ax), None if ar is None else _ptr(ar)))


def lst_get_t5_cuts(geom):
    """(xy, rz) float32 arrays of 1024: the quintuplet chi2 cuts in force per category."""
    xy = np.zeros(1024, np.float32)
    rz = np.zeros(1024, np.float32)
    _check(load_library().lst_get_t5_cuts(geom, _ptr(xy), _ptr(rz)))
    return xy, rz


def lst_t5_chi2_cuts():
    """(xy, rz) float32 arrays of 1024: the library's calibrated quintuplet cuts (host only)."""
    xy = np.zeros(1024, np.float32)
    rz = np.zeros(1024, np.float32)
    _check(load_library().lst_get_default_t5_cuts(_ptr(xy), _ptr(rz)))
    return xy, rz


def lst_set_track_extensions(geom, enable):
    _check(load_library().lst_set_track_extensions(geom, 1 if enable else 0))


def lst_get_extended_track_candidates(ev):
    """(types, offsets, hits, n_added, t3, attrs [n, 3]) of the extended collection."""
    lib = load_library()
    n, nh = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.lst_get_extended_track_candidates(ev, ctypes.byref(n), ctypes.byref(nh), None, None, None, None,
                                                 None, None))
    ty = np.zeros(n.value, np.int32)
    off = np.zeros(n.value + 1, np.int32)
    hits = np.zeros(nh.value, np.int32)
    na = np.zeros(n.value, np.int32)
    t3 = np.zeros(n.value, np.int32)
    at = np.zeros((n.value, 3), np.float32)
    _check(lib.lst_get_extended_track_candidates(ev, ctypes.byref(n), ctypes.byref(nh), _ptr(ty), _ptr(off),
                                                 _ptr(hits), _ptr(na), _ptr(t3), _ptr(at)))
    return ty, off, hits, na, t3, at


def lst_get_stage_objects(ev, stage):
    lib = load_library()
    n = ctypes.c_int32()
    _check(lib.lst_get_stage_objects(ev, int(stage), ctypes.byref(n), None, None, None))
    t = np.zeros((n.value, TUPLE_W[stage]), np.int32)
    f = np.zeros(n.value, np.int32)
    a = np.zeros((n.value, ATTR_W[stage]), np.float32)
    _check(lib.lst_get_stage_objects(ev, int(stage), ctypes.byref(n), _ptr(t), _ptr(f), _ptr(a)))
    return t, f, a


def lst_get_stage_counts(ev):
    c = np.zeros(8, np.int64)
    r = np.zeros(8, np.int64)
    _check(load_library().lst_get_stage_counts(ev, _ptr(c), _ptr(r)))
    return c, r


def lst_get_module_constants(geom, n_modules):
    out = np.zeros((n_modules, 4), np.float32)
    _check(load_library().lst_get_module_constants(geom, _ptr(out)))
    return out


def lst_release_event(ev):
    _check(load_library().lst_release_event(ev))


def lst_kernel_sites():
    lib = load_library()
    return [lib.lst_kernel_site_name(i).decode() for i in range(lib.lst_kernel_site_count())]


def lst_tiles():
    """[(name, lo, hi)] of the chain's tiles, in the order of the tile arrays."""
    lib = load_library()
    out = []
    for i in range(lib.lst_tile_count()):
        lo, hi = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.lst_tile_range(i, ctypes.byref(lo), ctypes.byref(hi)))
        out.append((lib.lst_tile_name(i).decode(), lo.value, hi.value))
    return out


def lst_get_tile_config(geom):
    n = load_library().lst_tile_count()
    a = np.zeros(n, np.int32)
    _check(load_library().lst_get_tile_config(geom, n, _ptr(a)))
    return a


def lst_set_tile_config(geom, tiles):
    a = np.ascontiguousarray(tiles, np.int32)
    _check(load_library().lst_set_tile_config(geom, int(a.size), _ptr(a)))


def lst_probe_valu(n_blocks, iters, out, stream=None):
    """Launches the VALU calibration kernel (see include/lst.h) into `out` (device float tensor)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(load_library().lst_probe_valu(int(n_blocks), int(iters), ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(stream)))


def lst_set_timed_site(site):
    _check(load_library().lst_set_timed_site(int(site)))


def lst_get_site_time(ev):
    ms = ctypes.c_float()
    _check(load_library().lst_get_site_time(ev, ctypes.byref(ms)))
    return float(ms.value)


def lst_get_launch_config(geom):
    """Threads per block of every launch site (0: fixed shape), as a list indexed by site."""
    lib = load_library()
    n = lib.lst_kernel_site_count()
    a = np.zeros(n, np.int32)
    _check(lib.lst_get_launch_config(geom, n, _ptr(a)))
    return [int(v) for v in a]


def lst_set_launch_config(geom, site_block):
    a = np.ascontiguousarray(site_block, np.int32)
    _check(load_library().lst_set_launch_config(geom, int(a.size), _ptr(a)))


def lst_autotune(geom, dev_events, workspace, caps=None, stream=None, reps=2):
    """Tunes the launch shapes on these events; returns the best time [ms] per launch site (-1: not tuned)."""
    lib = load_library()
    B = len(dev_events)
    descs = (lst_event_desc * B)(*[_event_desc(t) for t in dev_events])
    ca = _caps_array(caps)
    ms = np.zeros(lib.lst_kernel_site_count(), np.float32)
    _check(lib.lst_autotune(geom, B, ctypes.cast(descs, ctypes.c_void_p),
                            ctypes.cast(ca, ctypes.c_void_p) if ca is not None else None, _ptr(workspace),
                            int(workspace.numel()), stream, int(reps), _ptr(ms)))
    return ms


def _caps_array(caps):
    if caps is None:
        return None
    arr = (lst_capacity * len(caps))(*caps)
    return arr


def lst_batch_workspace_bytes(geom, n_hits, n_seeds, caps=None):
    nh = np.ascontiguousarray(n_hits, np.int32)
    ns = np.ascontiguousarray(n_seeds, np.int32)
    ca = _caps_array(caps)
    b = ctypes.c_size_t()
    _check(load_library().lst_batch_workspace_bytes(geom, int(nh.size), _ptr(nh), _ptr(ns),
                                                    ctypes.cast(ca, ctypes.c_void_p) if ca is not None else None,
                                                    ctypes.byref(b)))
    return int(b.value)


def lst_enqueue_batch(geom, dev_events, workspace, caps=None, stream=None):
    """Enqueues B events as one batch; returns (status, [event handles])."""
    B = len(dev_events)
    descs = (lst_event_desc * B)(*[_event_desc(t) for t in dev_events])
    ca = _caps_array(caps)
    outs = (ctypes.c_void_p * B)()
    st = load_library().lst_enqueue_batch(geom, B, ctypes.cast(descs, ctypes.c_void_p),
                                          ctypes.cast(ca, ctypes.c_void_p) if ca is not None else None,
                                          _ptr(workspace), int(workspace.numel()), stream,
                                          ctypes.cast(outs, ctypes.c_void_p))
    return st, [o for o in outs]


def lst_plan_workspace_bytes(geom, B, max_hits, max_seeds, cap=None):
    b = ctypes.c_size_t()
    _check(load_library().lst_plan_workspace_bytes(geom, int(B), int(max_hits), int(max_seeds),
                                                   ctypes.byref(cap) if cap is not None else None, ctypes.byref(b)))
    return int(b.value)


def lst_plan_create(geom, B, max_hits, max_seeds, workspace, cap=None, stream=None):
    h = ctypes.c_void_p()
    _check(load_library().lst_plan_create(geom, int(B), int(max_hits), int(max_seeds),
                                          ctypes.byref(cap) if cap is not None else None, _ptr(workspace),
                                          int(workspace.numel()), stream, ctypes.byref(h)))
    return h.value


def lst_plan_run(plan, dev_events, stream=None):
    """Replays the plan's graph for up to B events; returns (status, [event handles])."""
    n = len(dev_events)
    descs = (lst_event_desc * max(n, 1))(*[_event_desc(t) for t in dev_events])
    outs = (ctypes.c_void_p * max(n, 1))()
    st = load_library().lst_plan_run(plan, n, ctypes.cast(descs, ctypes.c_void_p), stream,
                                     ctypes.cast(outs, ctypes.c_void_p))
    return st, [outs[i] for i in range(n)]


def lst_plan_release(plan):
    _check(load_library().lst_plan_release(plan))


def lst_server_create(geom, n_streams, max_batch, pool):
    cfg = lst_server_config(int(n_streams), int(max_batch))
    h = ctypes.c_void_p()
    _check(load_library().lst_server_create(geom, ctypes.byref(cfg), _ptr(pool), int(pool.numel()),
                                            ctypes.byref(h)))
    return h.value


def lst_server_now(srv):
    t = ctypes.c_double()
    _check(load_library().lst_server_now(srv, ctypes.byref(t)))
    return t.value


def lst_server_submit(srv, dev_event, req_id, arrival_s, cap=None):
    d = _event_desc(dev_event)
    if cap is None:
        _check(load_library().lst_server_submit(srv, ctypes.byref(d), int(req_id), float(arrival_s)))
    else:
        _check(load_library().lst_server_submit_with_capacity(srv, ctypes.byref(d), ctypes.byref(cap), int(req_id),
                                                              float(arrival_s)))


def lst_server_reruns(srv):
    n = ctypes.c_int64()
    _check(load_library().lst_server_reruns(srv, ctypes.byref(n)))
    return int(n.value)


def lst_server_poll(srv, max_results=4096):
    buf = (lst_server_result * max_results)()
    n = ctypes.c_int32()
    _check(load_library().lst_server_poll(srv, ctypes.cast(buf, ctypes.c_void_p), int(max_results), ctypes.byref(n)))
    return [dict(id=buf[i].id, event=buf[i].event, arrival_s=buf[i].arrival_s, admit_s=buf[i].admit_s,
                 done_s=buf[i].done_s, status=buf[i].status) for i in range(n.value)]


def lst_server_pending(srv):
    q, r = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().lst_server_pending(srv, ctypes.byref(q), ctypes.byref(r)))
    return q.value, r.value


def lst_server_destroy(srv):
    _check(load_library().lst_server_destroy(srv))


# ------------------------------------------------------------- conveniences
class Geometry:
    """A detector uploaded to the device (owns the lst_geometry handle)."""

    def __init__(self, geom):
        m = geom.module_arrays()
        self.n_modules = int(geom.n_modules)
        self.handle = lst_load_geometry(m["subdet"], m["layer"], m["side"], m["type"], m["pos_lo"], m["pos_up"],
                                        m["lmin"], m["lmax"], geom.map_offsets, geom.map_targets)

    def module_constants(self):
        return lst_get_module_constants(self.handle, self.n_modules)

    def set_stub_precision(self, bits):
        """MD stubs stored in binary16 (16) or float (32, the default) by chains enqueued from now on."""
        lst_set_stub_precision(self.handle, bits)

    def set_impact_bound(self, d0_max):
        """Transverse impact-parameter bound of the selections [cm] (0.1 unless set)."""
        lst_set_impact_bound(self.handle, d0_max)

    def set_t5_cuts(self, xy=None, rz=None):
        """Quintuplet chi2 cuts per category for chains enqueued from now on (None: calibrated table)."""
        lst_set_t5_cuts(self.handle, xy, rz)

    def t5_cuts(self):
        """(xy, rz): the quintuplet chi2 cuts in force, 1024 categories each."""
        return lst_get_t5_cuts(self.handle)

    def set_track_extensions(self, enable=True):
        """Chains enqueued from now on end with (or without) the track-extension step."""
        lst_set_track_extensions(self.handle, enable)

    def launch_config(self):
        """{site name: threads per block} of the tunable launch sites."""
        return {n: b for n, b in zip(lst_kernel_sites(), lst_get_launch_config(self.handle)) if b}

    def set_launch_config(self, cfg):
        """Sets the launch shapes from {site name: threads per block} (other sites: default)."""
        names = lst_kernel_sites()
        unknown = set(cfg) - set(names)
        if unknown:
            raise LSTError(LST_E_INVALID, f"unknown launch sites {sorted(unknown)}")
        lst_set_launch_config(self.handle, [int(cfg.get(n, 0)) for n in names])

    def autotune(self, dev_events, reps=2, caps=None, stream=None):
        """Chooses the fastest launch shape per tunable site on these device events (one batch)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        nh = [int(t["x"].numel()) for t in dev_events]
        ns = [int(t["px"].numel()) for t in dev_events]
        ws = torch.empty(lst_batch_workspace_bytes(self.handle, nh, ns, caps), dtype=torch.uint8,
                         device=dev_events[0]["x"].device)
        ms = lst_autotune(self.handle, dev_events, ws, caps, stream, reps)
        del ws
        names = lst_kernel_sites()
        return {names[k]: (b, float(ms[k])) for k, b in enumerate(lst_get_launch_config(self.handle)) if b}

    def tile_config(self):
        """{tile name: value} of the chain's tiles."""
        return {n: int(v) for (n, _, _), v in zip(lst_tiles(), lst_get_tile_config(self.handle))}

    def set_tile_config(self, cfg):
        """Sets tiles from {tile name: value} (other tiles keep their values)."""
        names = [n for n, _, _ in lst_tiles()]
        unknown = set(cfg) - set(names)
        if unknown:
            raise LSTError(LST_E_INVALID, f"unknown tiles {sorted(unknown)}")
        cur = self.tile_config()
        cur.update({k: int(v) for k, v in cfg.items()})
        lst_set_tile_config(self.handle, [cur[n] for n in names])

    def autotune_tiles(self, dev_events, reps=2, caps=None, stream=None):
        """Chooses the fastest value per tile (whole-chain time over these device events, one batch);
        returns {tile: (value, ms)} of the tuned tiles."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        nh = [int(t["x"].numel()) for t in dev_events]
        ns = [int(t["px"].numel()) for t in dev_events]
        ws = torch.empty(lst_batch_workspace_bytes(self.handle, nh, ns, caps), dtype=torch.uint8,
                         device=dev_events[0]["x"].device)
        descs = (lst_event_desc * len(dev_events))(*[_event_desc(t) for t in dev_events])
        lib = load_library()
        ms = np.zeros(lib.lst_tile_count(), np.float32)
        ca = _caps_array(caps)
        _check(lib.lst_autotune_tiles(self.handle, len(dev_events), ctypes.cast(descs, ctypes.c_void_p),
                                      ctypes.cast(ca, ctypes.c_void_p) if ca is not None else None, _ptr(ws),
                                      int(ws.numel()), stream, int(reps), _ptr(ms)))
        del ws
        cfg = self.tile_config()
        return {n: (cfg[n], float(m)) for (n, _, _), m in zip(lst_tiles(), ms) if m >= 0}

    def save_launch_config(self, path):
        """Launch shapes and tiles to a JSON file ({site: threads per block, "tiles": {...}})."""
        import json
        with open(path, "w") as fh:
            json.dump({**self.launch_config(), "tiles": self.tile_config()}, fh, indent=1, sort_keys=True)

    def load_launch_config(self, path):
        import json
        with open(path) as fh:
            cfg = json.load(fh)
        tiles = cfg.pop("tiles", None)
        self.set_launch_config(cfg)
        if tiles:
            self.set_tile_config(tiles)

    def close(self):
        if self.handle:
            lst_release_geometry(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upload_event(ev, device="cuda"):
    """Copies an event's arrays (numpy) to device tensors in the C ABI's layout."""
    import torch
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    i = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(device)
    return dict(x=f(ev.x), y=f(ev.y), z=f(ev.z), module=i(ev.module), sensor=i(ev.sensor),
                px=f(ev.px), py=f(ev.py), pz=f(ev.pz), q=i(ev.q), hits4=i(np.asarray(ev.hits4).reshape(-1)))


class EventResult:
    """A built event: the library's handle plus the workspace it lives in."""

    def __init__(self, handle, workspace, status):
        self.handle, self.workspace, self.status = handle, workspace, status

    def track_candidates(self):
        return lst_get_track_candidates(self.handle)

    def extended_track_candidates(self):
        return lst_get_extended_track_candidates(self.handle)

    def stage(self, stage):
        return lst_get_stage_objects(self.handle, stage)

    def counts(self):
        return lst_get_stage_counts(self.handle)

    def close(self):
        if self.handle:
            lst_release_event(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def alloc_workspace(geom, n_hits, n_seeds, cap=None, device="cuda"):
    import torch
    nb = lst_workspace_bytes(geom.handle, n_hits, n_seeds, cap)
    return torch.empty(nb, dtype=torch.uint8, device=device)


def run_batch(geom, dev_events, caps=None, workspace=None, stream=None):
    """Builds B events in one batch and waits; returns one EventResult per event."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    nh = [int(t["x"].numel()) for t in dev_events]
    ns = [int(t["px"].numel()) for t in dev_events]
    need = lst_batch_workspace_bytes(geom.handle, nh, ns, caps)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev_events[0]["x"].device)
    st, hs = lst_enqueue_batch(geom.handle, dev_events, workspace, caps, stream)
    _check(st)
    out = []
    for h in hs:
        s = lst_event_wait(h)
        out.append(EventResult(h, workspace, s))
    bad = [r.status for r in out if r.status != LST_OK]
    if bad:
        msg = lst_last_error()
        for r in out:
            r.close()
        raise LSTError(bad[0], msg)
    return out


class Plan:
    """A captured batch chain (HIP graph) over B slots in its own workspace."""

    def __init__(self, geom, B, max_hits, max_seeds, cap=None, device="cuda", stream=None):
        import torch
        self.B = B
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self.workspace = torch.empty(lst_plan_workspace_bytes(geom.handle, B, max_hits, max_seeds, cap),
                                     dtype=torch.uint8, device=device)
        self.handle = lst_plan_create(geom.handle, B, max_hits, max_seeds, self.workspace, cap, stream)

    def run(self, dev_events, wait=True):
        st, hs = lst_plan_run(self.handle, dev_events, self.stream)
        _check(st)
        res = [EventResult(h, self.workspace, LST_OK) for h in hs]
        if wait:
            for r in res:
                r.status = lst_event_wait(r.handle)
        return res

    def close(self):
        if self.handle:
            lst_plan_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The library's serving loop with a device pool (a torch uint8 tensor) of pool_bytes."""

    def __init__(self, geom, n_streams, max_batch, pool_bytes, device="cuda"):
        import torch
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        torch.cuda.synchronize()
        self.handle = lst_server_create(geom.handle, n_streams, max_batch, self.pool)

    def now(self):
        return lst_server_now(self.handle)

    def submit(self, dev_event, req_id, arrival_s=0.0, cap=None):
        lst_server_submit(self.handle, dev_event, req_id, arrival_s, cap)

    def reruns(self):
        """Requests run again after a capacity overflow."""
        return lst_server_reruns(self.handle)

    def poll(self):
        return lst_server_poll(self.handle)

    def pending(self):
        return lst_server_pending(self.handle)

    def drain(self, n_expected, on_result, timeout_s=120.0):
        """Polls until n_expected results arrived; on_result(result dict) must release result['event']."""
        import time
        got = 0
        t_end = time.monotonic() + timeout_s
        while got < n_expected:
            rs = self.poll()
            for r in rs:
                on_result(r)
            got += len(rs)
            if not rs:
                if time.monotonic() > t_end:
                    raise TimeoutError(f"server drained {got} of {n_expected} results")
                time.sleep(0.0005)
        return got

    def close(self):
        if self.handle:
            lst_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_event(geom, dev_event, cap=None, workspace=None, stream=None, grow=True):
    """Builds one event; on LST_E_CAPACITY grows the capacities to the reported needs and reruns."""
    import torch
    n_hits, n_seeds = int(dev_event["x"].numel()), int(dev_event["px"].numel())
    if cap is None:
        cap = lst_default_capacity(n_hits, n_seeds)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    for _ in range(4):
        need = lst_workspace_bytes(geom.handle, n_hits, n_seeds, cap)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=dev_event["x"].device)
        st, h = lst_build_event(geom.handle, dev_event, workspace, cap, stream)
        if st == LST_E_CAPACITY and grow:
            _, req = lst_get_stage_counts(h)
            lst_release_event(h)
            names = ["md", "ls", "t3", "t5", None, "pt3", "pt5"]
            for k, nm in enumerate(names):
                if nm and req[k] > getattr(cap, nm):
                    setattr(cap, nm, int(req[k] * 1.25) + 1024)
            continue
        if st != LST_OK:
            msg = lst_last_error()
            if h:
                lst_release_event(h)
            raise LSTError(st, msg)
        return EventResult(h, workspace, st)
    raise LSTError(LST_E_CAPACITY, "capacities kept growing")
