"""CPU oracle of the adaptive density hierarchy -- test infrastructure.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The device library never does, and the two
share no code.

``ahf_oracle.c`` is the double-precision definition (see its header for the
readings of the paper it follows); ``brute.py`` is an independent dense
brute force for tiny inputs used to pin it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ahf_oracle.c")
LIB = os.path.join(HERE, "libahf_oracle.so")
# the same source built for the host it runs on (-O3 -march=native), used only
# to time the oracle as a CPU baseline
LIB_NATIVE = os.path.join(HERE, "libahf_oracle_native.so")


def build_library(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with the host C compiler (gcc)."""
    out = LIB_NATIVE if native else LIB
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        tmp = out + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *opt, "-std=c11", "-Wall", "-shared", "-fPIC", SRC,
                        "-o", tmp, "-lm"], check=True)
        os.replace(tmp, out)
    return out


_libs = {}

_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib(native: bool = False):
    if native not in _libs:
        path = LIB_NATIVE if native else LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build_library(force=True, native=native)
        L = C.CDLL(path)
        L.orc_build.restype = C.c_int
        L.orc_build.argtypes = [C.c_uint64, _u32p, _u32p, _u32p, _f32p, _f32p, _f32p,
                                C.c_void_p, C.c_double, C.c_int, C.c_double, C.c_double,
                                C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_num_levels.restype = C.c_int
        L.orc_num_levels.argtypes = [C.c_void_p]
        L.orc_order.restype = C.POINTER(C.c_uint32)
        L.orc_order.argtypes = [C.c_void_p]
        L.orc_level_sizes.argtypes = [C.c_void_p, C.c_int, _u64p]
        L.orc_level_cells.argtypes = [C.c_void_p, C.c_int, _u64p, _u32p, _u32p, _u8p, _i32p, _f64p]
        L.orc_level_field.argtypes = [C.c_void_p, C.c_int, _u64p, _f64p, _u8p]
        L.orc_level_totals.argtypes = [C.c_void_p, C.c_int, _f64p]
        L.orc_level_patches.argtypes = [C.c_void_p, C.c_int, _i32p, _u64p, _u64p, _f64p]
        L.orc_probe_create.restype = C.c_void_p
        L.orc_probe_create.argtypes = [C.c_uint64, _u32p, _u32p, _u32p, _f32p, _f32p, _f32p,
                                       C.c_void_p, C.c_double, C.c_int, C.c_double, C.c_double,
                                       C.c_int]
        L.orc_probe_free.argtypes = [C.c_void_p]
        L.orc_probe_cell.restype = C.c_int
        L.orc_probe_cell.argtypes = [C.c_void_p, C.c_int, C.c_uint64, _i64p, C.POINTER(C.c_double)]
        L.orc_morton.restype = C.c_uint64
        L.orc_morton.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_int]
        _libs[native] = L
    return _libs[native]


def _arrays(p):
    X = np.ascontiguousarray(p.X, dtype=np.uint32)
    Y = np.ascontiguousarray(p.Y, dtype=np.uint32)
    Z = np.ascontiguousarray(p.Z, dtype=np.uint32)
    fx = np.ascontiguousarray(p.fx, dtype=np.float32)
    fy = np.ascontiguousarray(p.fy, dtype=np.float32)
    fz = np.ascontiguousarray(p.fz, dtype=np.float32)
    m = None if getattr(p, "mass", None) is None else np.ascontiguousarray(p.mass, dtype=np.float32)
    return X, Y, Z, fx, fy, fz, m


class Level:
    """One level of the oracle hierarchy as numpy arrays."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def build(p, g=None, dom_ref=None, ref_ref=None, max_levels=None, connectivity=26,
          labels=True, mass_scalar=1.0, density=False, native=False):
    """Run the oracle on a particle set (anything with X, Y, Z, fx, fy, fz and
    optionally mass attributes; parameters default to the object's own).
    density: refine on the TSC particle number of a cell instead of its
    particle count; native: the -O3 -march=native build of the same source.
    Returns (levels, order)."""
    L = lib(native)
    X, Y, Z, fx, fy, fz, m = _arrays(p)
    g = p.g if g is None else g
    dom_ref = p.dom_ref if dom_ref is None else dom_ref
    ref_ref = p.ref_ref if ref_ref is None else ref_ref
    max_levels = p.max_levels if max_levels is None else max_levels
    h = C.c_void_p()
    rc = L.orc_build(len(X), X, Y, Z, fx, fy, fz,
                     None if m is None else m.ctypes.data_as(C.c_void_p),
                     float(mass_scalar), int(g), float(dom_ref), float(ref_ref),
                     int(max_levels), int(connectivity), int(bool(labels)), int(bool(density)),
                     C.byref(h))
    if rc != 0:
        raise ValueError(f"oracle build failed with code {rc}")
    try:
        nlev = L.orc_num_levels(h)
        order = np.ctypeslib.as_array(L.orc_order(h), shape=(len(X),)).copy() if len(X) else \
            np.zeros(0, np.uint32)
        levels = []
        for lv in range(nlev):
            sz = np.zeros(5, np.uint64)
            L.orc_level_sizes(h, lv, sz)
            nS, nE, nP, npatch, b = (int(v) for v in sz)
            key = np.zeros(nS, np.uint64); cnt = np.zeros(nS, np.uint32)
            start = np.zeros(nS, np.uint32); flag = np.zeros(nS, np.uint8)
            patch = np.zeros(nS, np.int32); pmass = np.zeros(nS, np.float64)
            L.orc_level_cells(h, lv, key, cnt, start, flag, patch, pmass)
            ekey = np.zeros(nE, np.uint64); emass = np.zeros(nE, np.float64)
            ghost = np.zeros(nE, np.uint8)
            L.orc_level_field(h, lv, ekey, emass, ghost)
            tot = np.zeros(2, np.float64)
            L.orc_level_totals(h, lv, tot)
            pp = np.zeros(npatch, np.int32); pnc = np.zeros(npatch, np.uint64)
            pnp = np.zeros(npatch, np.uint64); pm = np.zeros(npatch, np.float64)
            L.orc_level_patches(h, lv, pp, pnc, pnp, pm)
            levels.append(Level(level=lv, bits=b, n_particles=nP, cell_key=key,
                                cell_count=cnt, cell_start=start, cell_flag=flag,
                                cell_patch=patch, cell_pmass=pmass, field_key=ekey,
                                field_mass=emass, field_ghost=ghost,
                                total_cell_mass=tot[0], total_particle_mass=tot[1],
                                n_patches=npatch, patch_parent=pp, patch_ncells=pnc,
                                patch_nparticles=pnp, patch_mass=pm))
        return levels, order
    finally:
        L.orc_free(h)


class Probe:
    """Single-cell questions answered from the definition on inputs too large
    for ``build`` (sorts the particles once)."""

    def __init__(self, p, g=None, dom_ref=None, ref_ref=None, max_levels=None,
                 mass_scalar=1.0):
        L = lib()
        self._keep = _arrays(p)
        X, Y, Z, fx, fy, fz, m = self._keep
        self.g = p.g if g is None else g
        self.max_levels = p.max_levels if max_levels is None else max_levels
        self._h = L.orc_probe_create(
            len(X), X, Y, Z, fx, fy, fz, None if m is None else m.ctypes.data_as(C.c_void_p),
            float(mass_scalar), int(self.g), float(p.dom_ref if dom_ref is None else dom_ref),
            float(p.ref_ref if ref_ref is None else ref_ref), int(self.max_levels))
        if not self._h:
            raise ValueError("oracle probe creation failed")

    def cell(self, level: int, key: int) -> dict:
        out = np.zeros(5, np.int64)
        m = C.c_double()
        rc = lib().orc_probe_cell(self._h, int(level), C.c_uint64(int(key)), out, C.byref(m))
        if rc != 0:
            raise ValueError("bad probe")
        return dict(in_S=bool(out[0]), in_E=bool(out[1]), count=int(out[2]),
                    start=int(out[3]), flag=bool(out[4]), mass=m.value)

    def close(self):
        if self._h:
            lib().orc_probe_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def morton(x: int, y: int, z: int, bits: int) -> int:
    return int(lib().orc_morton(x, y, z, bits))
