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
        lib.orc_geom_set_pt_plain.argtypes = [vp, ctypes.c_int]
        lib.orc_t5_cuts.argtypes = [vp, vp, vp]
        i32 = ctypes.c_int
        lib.orc_probe_md.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_probe_ls.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_probe_t3.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_probe_t5.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        f32, f64_ = ctypes.c_float, ctypes.c_double
        lib.orc_probe_pt.argtypes = [vp, i32, vp, vp, vp, vp, f32, f32, f32, i32, f64_, f64_, vp, vp, vp, vp, vp]
        lib.orc_probe_near.argtypes = [f64_] * 7
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

    def set_pt_plain(self, on=True):
        """Seed search over every (seed, object) pair with no window pre-test (same results)."""
        self.lib.orc_geom_set_pt_plain(ctypes.c_void_p(self.handle), 1 if on else 0)

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


# --------------------------------------------------------- selection probes
class Probe:
    """One selection evaluated on hand-placed hits (test instrumentation).

    ok: the predicate's decision; cuts: every cut it evaluated, in order, as
    (quantity, bound, kind) with kind 0 for "passes when quantity <= bound"
    and 1 for "passes when quantity > bound"; attr: what the stage reports."""

    def __init__(self, ok, q, b, kind, n, attr=None, extra=None):
        self.ok = bool(ok)
        self.cuts = [(float(q[k]), float(b[k]), int(kind[k])) for k in range(n)]
        self.attr = attr
        self.extra = extra

    def passes(self, k):
        q, b, kind = self.cuts[k]
        return q <= b if kind == 0 else q > b

    def failing(self):
        return [k for k in range(len(self.cuts)) if not self.passes(k)]


def _hits(xyz, n):
    a = np.ascontiguousarray(np.asarray(xyz, np.float32).reshape(n, 3))
    return [np.ascontiguousarray(a[:, i]) for i in range(3)]


def _trace():
    return np.zeros(48, np.float64), np.zeros(48, np.float64), np.zeros(48, np.int32), ctypes.c_int(0)


def probe_md(og, module, lower, upper):
    """MD selection of a lower and an upper hit (x, y, z) in one module."""
    x, y, z = _hits([lower, upper], 2)
    q, b, k, n = _trace()
    ok = og.lib.orc_probe_md(ctypes.c_void_p(og.handle), int(module), _p(x), _p(y), _p(z), _p(q), _p(b), _p(k),
                             ctypes.byref(n))
    return Probe(ok, q, b, k, n.value)


def probe_ls(og, modules, hits):
    """Segment selection of MD 0 (hits 0, 1; inner) and MD 1 (hits 2, 3); attr = (beta_in, beta_out)."""
    x, y, z = _hits(hits, 4)
    m = np.ascontiguousarray(modules, np.int32)
    beta = np.zeros(2, np.float64)
    q, b, k, n = _trace()
    ok = og.lib.orc_probe_ls(ctypes.c_void_p(og.handle), _p(m), _p(x), _p(y), _p(z), _p(beta), _p(q), _p(b), _p(k),
                             ctypes.byref(n))
    return Probe(ok, q, b, k, n.value, attr=beta)


def probe_t3(og, modules, hits):
    """Triplet selection of MDs 0, 1, 2 (hits 2k, 2k + 1); attr = (kappa, dkappa, chi2_rz, lambda)."""
    x, y, z = _hits(hits, 6)
    m = np.ascontiguousarray(modules, np.int32)
    attr = np.zeros(4, np.float64)
    q, b, k, n = _trace()
    ok = og.lib.orc_probe_t3(ctypes.c_void_p(og.handle), _p(m), _p(x), _p(y), _p(z), _p(attr), _p(q), _p(b), _p(k),
                             ctypes.byref(n))
    return Probe(ok, q, b, k, n.value, attr=attr)


def probe_t5(og, modules, hits):
    """Quintuplet selection of MDs 0-4 (triplets (0, 1, 2) and (2, 3, 4)); extra = the two T3 decisions."""
    x, y, z = _hits(hits, 10)
    m = np.ascontiguousarray(modules, np.int32)
    attr = np.zeros(8, np.float64)
    t3ok = np.zeros(2, np.int32)
    q, b, k, n = _trace()
    ok = og.lib.orc_probe_t5(ctypes.c_void_p(og.handle), _p(m), _p(x), _p(y), _p(z), _p(t3ok), _p(attr), _p(q),
                             _p(b), _p(k), ctypes.byref(n))
    return Probe(ok, q, b, k, n.value, attr=attr, extra=t3ok)


def probe_pt(og, modules, pixel_hits, md_hits, seed, kT, dkT):
    """pT3 / pT5 selection: seed = (px, py, pz, charge) with four pixel hits, outer object on
    len(modules) MDs (hits 2k, 2k + 1 of md_hits), its curvature kT and error dkT;
    attr = (chi2_xy, chi2_rz, score)."""
    kk = len(modules)
    x, y, z = _hits(list(pixel_hits) + list(md_hits), 4 + 2 * kk)
    m = np.ascontiguousarray(modules, np.int32)
    attr = np.zeros(3, np.float64)
    q, b, k, n = _trace()
    px, py, pz, ch = seed
    ok = og.lib.orc_probe_pt(ctypes.c_void_p(og.handle), kk, _p(m), _p(x), _p(y), _p(z), float(px), float(py),
                             float(pz), int(ch), float(kT), float(dkT), _p(attr), _p(q), _p(b), _p(k), ctypes.byref(n))
    return Probe(ok, q, b, k, n.value, attr=attr)


def probe_near(og, a, b, D):
    """Section 2.5's near test between directions a, b = (dx, dy, lambda) at distance D."""
    return bool(og.lib.orc_probe_near(*(float(v) for v in a), *(float(v) for v in b), float(D)))
