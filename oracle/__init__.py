"""CPU oracle of the Line Segment Tracking chain: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never links, loads or
calls it.  See ``lst_oracle.c`` for the selections and their citations.

``build()`` compiles two shared libraries from the same C source with
``gcc -O2 -ffp-contract=off``: the FP32 oracle and its FP64 shadow.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lst_oracle.c")
BUILD = os.path.join(HERE, "_build")
LIBS = {False: os.path.join(BUILD, "liblst_oracle32.so"), True: os.path.join(BUILD, "liblst_oracle64.so")}

ST_MD, ST_LS, ST_T3, ST_T5, ST_PLS, ST_PT3, ST_PT5, ST_TC = range(8)
STAGE_NAMES = ["MD", "LS", "T3", "T5", "pLS", "pT3", "pT5", "TC"]
TUPLE_W = [2, 4, 6, 10, 1, 7, 11, 0]
ATTR_W = [0, 2, 4, 8, 5, 3, 3, 0]
# timed steps of a run: set-up, the eight stages (with their duplicate removal
# and cross-cleaning), track extensions
STEP_NAMES = ["setup"] + STAGE_NAMES + ["ext"]


def build(force=True):
    """Compile the FP32 oracle and the FP64 shadow (gcc, no FMA contraction)."""
    os.makedirs(BUILD, exist_ok=True)
    for f64, out in LIBS.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99",
               "-Wall", "-o", out + ".tmp", SRC, "-lm"]
        if f64:
            cmd.insert(1, "-DORACLE_F64")
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


_LIBS = {}


def _lib(f64=False):
    if f64 not in _LIBS:
        if not os.path.exists(LIBS[f64]):
            build(force=False)
        lib = ctypes.CDLL(LIBS[f64])
        vp = ctypes.c_void_p
        lib.orc_geom_create.restype = vp
        lib.orc_run.restype = vp
        lib.orc_run_brute.restype = vp
        lib.orc_count.restype = ctypes.c_int
        lib.orc_count.argtypes = [vp, ctypes.c_int]
        lib.orc_stage.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        lib.orc_tc.argtypes = [vp, vp, vp, vp]
        lib.orc_tc_hit_count.argtypes = [vp]
        lib.orc_ext_hit_count.argtypes = [vp]
        lib.orc_ext.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.orc_step_seconds.argtypes = [vp, ctypes.c_int]
        lib.orc_step_seconds.restype = ctypes.c_double
        lib.orc_border_count.argtypes = [vp, ctypes.c_int]
        lib.orc_border.argtypes = [vp, ctypes.c_int, vp, vp]
        lib.orc_free.argtypes = [vp]
        lib.orc_geom_free.argtypes = [vp]
        lib.orc_geom_set_d0max.argtypes = [vp, ctypes.c_double]
        lib.orc_geom_set_stub16.argtypes = [vp, ctypes.c_int]
        lib.orc_round_half.argtypes = [ctypes.c_double]
        lib.orc_round_half.restype = ctypes.c_double
        lib.orc_geom_set_t5_cuts.argtypes = [vp, vp, vp]
        lib.orc_t5_cuts.argtypes = [vp, vp, vp]
        lib.orc_module_consts.argtypes = [vp, vp]
        lib.orc_module_consts_f64.argtypes = [vp, vp]
        _LIBS[f64] = lib
    return _LIBS[f64]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleGeometry:
    """The oracle's copy of a detector (module table + module map)."""

    def __init__(self, geom, f64=False, d0_max=None, stub16=False):
        """d0_max: transverse impact-parameter bound of the selections [cm] (default 0.1);
        stub16: MD stubs kept in binary16."""
        self.f64 = f64
        self.lib = _lib(f64)
        m = geom.module_arrays()
        self._keep = [np.ascontiguousarray(m[k], dtype=np.int32) for k in ("subdet", "layer", "side", "type")]
        self._keep += [np.ascontiguousarray(m[k], dtype=np.float32) for k in ("pos_lo", "pos_up", "lmin", "lmax")]
        off = np.ascontiguousarray(geom.map_offsets, dtype=np.int32)
        tgt = np.ascontiguousarray(geom.map_targets, dtype=np.int32)
        self.n_modules = int(geom.n_modules)
        self.handle = self.lib.orc_geom_create(ctypes.c_int(self.n_modules), *[_p(a) for a in self._keep[:4]],
                                               *[_p(a) for a in self._keep[4:]], ctypes.c_int(int(tgt.size)),
                                               _p(off), _p(tgt))
        if d0_max is not None:
            self.lib.orc_geom_set_d0max(ctypes.c_void_p(self.handle), ctypes.c_double(float(d0_max)))
        if stub16:
            self.lib.orc_geom_set_stub16(ctypes.c_void_p(self.handle), 1)

    def set_t5_cuts(self, xy=None, rz=None):
        """Quintuplet chi2 cuts of the 1024 categories (None: the calibrated table)."""
        ax = None if xy is None else np.ascontiguousarray(np.broadcast_to(xy, (1024,)), np.float64)
        ar = None if rz is None else np.ascontiguousarray(np.broadcast_to(rz, (1024,)), np.float64)
        self.lib.orc_geom_set_t5_cuts(ctypes.c_void_p(self.handle), None if ax is None else _p(ax),
                                      None if ar is None else _p(ar))

    def t5_cuts(self):
        """(xy, rz): the quintuplet chi2 cuts in force, per category (1024 each)."""
        xy = np.zeros(1024, np.float64)
        rz = np.zeros(1024, np.float64)
        self.lib.orc_t5_cuts(ctypes.c_void_p(self.handle), _p(xy), _p(rz))
        return xy, rz

    def module_consts(self, as_f64=False):
        """(n_modules, 4) array of W, A1, A2, A3 (rounded to the oracle's precision unless as_f64)."""
        if as_f64:
            out = np.zeros((self.n_modules, 4), np.float64)
            self.lib.orc_module_consts_f64(ctypes.c_void_p(self.handle), _p(out))
        else:
            out = np.zeros((self.n_modules, 4), np.float64 if self.f64 else np.float32)
            self.lib.orc_module_consts(ctypes.c_void_p(self.handle), _p(out))
        return out

    def __del__(self):
        try:
            self.lib.orc_geom_free(ctypes.c_void_p(self.handle))
        except Exception:
            pass


class OracleResult:
    def __init__(self, lib, handle, f64, n_hits):
        self.lib, self.handle, self.f64, self.n_hits = lib, handle, f64, n_hits

    def count(self, stage):
        return int(self.lib.orc_count(ctypes.c_void_p(self.handle), stage))

    def stage(self, stage):
        """(tuples [n, w] int32, flags [n] int32, attrs [n, a] float) of one stage."""
        n = self.count(stage)
        t = np.zeros((n, TUPLE_W[stage]), np.int32)
        f = np.zeros(n, np.int32)
        a = np.zeros((n, ATTR_W[stage]), np.float64 if self.f64 else np.float32)
        self.lib.orc_stage(ctypes.c_void_p(self.handle), stage, _p(t), _p(f), _p(a))
        return t, f, a

    def tc(self):
        n = self.count(ST_TC)
        nh = int(self.lib.orc_tc_hit_count(ctypes.c_void_p(self.handle)))
        ty = np.zeros(n, np.int32)
        off = np.zeros(n + 1, np.int32)
        hits = np.zeros(nh, np.int32)
        self.lib.orc_tc(ctypes.c_void_p(self.handle), _p(ty), _p(off), _p(hits))
        return ty, off, hits

    def extensions(self):
        """Track extensions of the TCs, in TC order: (n_added [n], t3 index [n] (-1: none),
        attrs [n, 3] (chi2_xy, chi2_rz, kappa), offsets [n + 1], hits) of the extended collection."""
        n = self.count(ST_TC)
        nh = int(self.lib.orc_ext_hit_count(ctypes.c_void_p(self.handle)))
        na = np.zeros(n, np.int32)
        t3 = np.zeros(n, np.int32)
        at = np.zeros((n, 3), np.float64 if self.f64 else np.float32)
        off = np.zeros(n + 1, np.int32)
        hits = np.zeros(nh, np.int32)
        self.lib.orc_ext(ctypes.c_void_p(self.handle), _p(na), _p(t3), _p(at), _p(off), _p(hits))
        return na, t3, at, off, hits

    def step_seconds(self):
        """{step name: wall seconds} of the run, measured by the oracle on its own thread."""
        return {n: float(self.lib.orc_step_seconds(ctypes.c_void_p(self.handle), k))
                for k, n in enumerate(STEP_NAMES)}

    def border(self, stage):
        n = int(self.lib.orc_border_count(ctypes.c_void_p(self.handle), stage))
        t = np.zeros((n, max(TUPLE_W[stage], 1)), np.int32)
        acc = np.zeros(n, np.int32)
        if n:
            self.lib.orc_border(ctypes.c_void_p(self.handle), stage, _p(t), _p(acc))
        return t, acc

    def __del__(self):
        try:
            self.lib.orc_free(ctypes.c_void_p(self.handle))
        except Exception:
            pass


def _event_args(ev):
    a = dict(x=np.ascontiguousarray(ev.x, np.float32), y=np.ascontiguousarray(ev.y, np.float32),
             z=np.ascontiguousarray(ev.z, np.float32), module=np.ascontiguousarray(ev.module, np.int32),
             sensor=np.ascontiguousarray(ev.sensor, np.int32), px=np.ascontiguousarray(ev.px, np.float32),
             py=np.ascontiguousarray(ev.py, np.float32), pz=np.ascontiguousarray(ev.pz, np.float32),
             q=np.ascontiguousarray(ev.q, np.int32), hits4=np.ascontiguousarray(ev.hits4, np.int32).reshape(-1, 4))
    return a


def run(ogeom, ev, last=ST_TC):
    """Run the staged oracle on an event up to stage `last`."""
    a = _event_args(ev)
    h = ogeom.lib.orc_run(ctypes.c_void_p(ogeom.handle), ctypes.c_int(ev.n_hits), _p(a["x"]), _p(a["y"]),
                          _p(a["z"]), _p(a["module"]), _p(a["sensor"]), ctypes.c_int(ev.n_seeds), _p(a["px"]),
                          _p(a["py"]), _p(a["pz"]), _p(a["q"]), _p(a["hits4"]), ctypes.c_int(last))
    return OracleResult(ogeom.lib, h, ogeom.f64, ev.n_hits)


def run_brute(ogeom, ev):
    """Brute-force closure of MD, LS, T3, T5 and T5 duplicate removal (tiny events only)."""
    a = _event_args(ev)
    counts = np.zeros(5, np.int32)
    h = ogeom.lib.orc_run_brute(ctypes.c_void_p(ogeom.handle), ctypes.c_int(ev.n_hits), _p(a["x"]), _p(a["y"]),
                                _p(a["z"]), _p(a["module"]), _p(a["sensor"]), _p(counts))
    return OracleResult(ogeom.lib, h, ogeom.f64, ev.n_hits), counts
