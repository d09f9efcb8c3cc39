"""Python binding of libahf.so (ctypes; argument marshalling only).

Every step of the hierarchy runs in the library's HIP kernels.  PyTorch only
provides device memory (input tensors) and streams.  If the library has not
been built, every call raises: there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libahf.so")

AHF_OK, AHF_PENDING = 0, 1
AHF_EINVAL, AHF_ENOMEM, AHF_EDEVICE, AHF_ELIMIT = -1, -2, -3, -4
AHF_EBUSY, AHF_ENOTFOUND, AHF_ECANCELED = -5, -6, -7
AHF_NO_LABELS = 1
AHF_SUBSTRUCTURE = 2
AHF_DENSITY_CRITERION = 4

# every symbol declared in include/ahf.h
EXPORTS = [
    "ahf_last_error", "ahf_ctx_create", "ahf_ctx_destroy", "ahf_build_hierarchy",
    "ahf_label_refinements", "ahf_hierarchy_num_levels", "ahf_level_get",
    "ahf_hierarchy_order", "ahf_hierarchy_timings", "ahf_hierarchy_free",
    "ahf_ctx_set_profiling", "ahf_ctx_profile_only", "ahf_ctx_kernel_time", "ahf_hierarchy_query_label",
    "ahf_server_create", "ahf_submit", "ahf_poll", "ahf_wait", "ahf_query_label",
    "ahf_release", "ahf_ticket_times", "ahf_server_get_stats", "ahf_server_destroy",
    "ahf_classify_substructure", "ahf_hierarchy_structures",
    "ahf_hierarchy_query_label_static", "ahf_ctx_set_tuning", "ahf_ctx_get_tuning",
    "ahf_ctx_set_planning", "ahf_hierarchy_build_info",
    "ahf_batch_create", "ahf_batch_run", "ahf_batch_wait", "ahf_batch_status",
    "ahf_batch_hierarchy", "ahf_batch_destroy",
    "ahf_find_halos", "ahf_halos_get", "ahf_halos_free",
]


class AhfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ahf error {code}: {msg}")
        self.code = code


class CtxDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("device", C.c_int32), ("alloc", C.c_void_p),
                ("free", C.c_void_p), ("user", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("dom_grid_log2", C.c_uint32),
                ("dom_ref", C.c_double), ("ref_ref", C.c_double), ("max_levels", C.c_uint32),
                ("connectivity", C.c_uint32), ("flags", C.c_uint32)]


class Particles(C.Structure):
    _fields_ = [("n", C.c_uint64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("fx", C.c_void_p), ("fy", C.c_void_p), ("fz", C.c_void_p),
                ("mass", C.c_void_p), ("mass_scalar", C.c_double)]


class LevelView(C.Structure):
    _fields_ = [("level", C.c_uint32), ("bits", C.c_uint32), ("n_cells", C.c_uint64),
                ("n_refined", C.c_uint64), ("n_particles", C.c_uint64),
                ("n_bricks", C.c_uint64), ("n_patches", C.c_uint64),
                ("cell_key", C.c_void_p), ("cell_start", C.c_void_p),
                ("cell_count", C.c_void_p), ("cell_refined", C.c_void_p),
                ("cell_patch", C.c_void_p), ("brick_key", C.c_void_p),
                ("brick_cell", C.c_void_p), ("brick_mass", C.c_void_p),
                ("patch_parent", C.c_void_p), ("patch_ncells", C.c_void_p),
                ("patch_nparticles", C.c_void_p), ("patch_mass", C.c_void_p),
                ("total_cell_mass", C.c_double), ("total_particle_mass", C.c_double),
                ("patch_struct", C.c_void_p)]


class Structures(C.Structure):
    _fields_ = [("n_structures", C.c_uint64), ("host", C.c_void_p), ("level", C.c_void_p),
                ("patch", C.c_void_p), ("depth", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("heavy_level0", C.c_uint32),
                ("heavy_level1", C.c_uint32), ("heavy_deeper", C.c_uint32),
                ("batch_level1", C.c_uint32), ("sort_skip_digits", C.c_int32)]


class BuildInfo(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("planned", C.c_uint32), ("replanned", C.c_uint32),
                ("host_waits", C.c_uint32), ("device_bytes", C.c_uint64),
                ("sort_key_bits", C.c_uint32), ("sort_passes", C.c_uint32)]


class HaloParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("delta_vir", C.c_double), ("G", C.c_double),
                ("max_iter", C.c_uint32), ("large_from", C.c_uint32)]


class HalosView(C.Structure):
    _fields_ = [("n_halos", C.c_uint64), ("leaf", C.c_void_p), ("centre", C.c_void_p),
                ("radius", C.c_void_p), ("cand_offset", C.c_void_p), ("cand_count", C.c_void_p),
                ("cand", C.c_void_p), ("member_count", C.c_void_p), ("member", C.c_void_p),
                ("r_vir", C.c_void_p), ("m_vir", C.c_void_p), ("vel", C.c_void_p),
                ("iterations", C.c_void_p)]


class ServerDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_streams", C.c_uint32),
                ("max_queue", C.c_uint32), ("flags", C.c_uint32), ("hbm_budget", C.c_uint64)]


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("submitted", "completed", "failed", "evicted",
                                          "released", "queued", "running", "resident",
                                          "bytes_in_use", "bytes_peak", "bytes_results")]


# device memory callbacks of ahf_ctx_desc
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class TorchMemory:
    """Device memory from PyTorch's caching allocator, for ahf_ctx_desc: the
    library's hierarchies and scratch space are then PyTorch-owned HBM, taken
    and given back in the order of the stream the library passes."""

    def __init__(self):
        import torch
        raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc
        raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete

        def alloc(user, nbytes, stream):
            try:
                return raw_alloc(int(nbytes), int(stream or 0))
            except Exception:  # out of memory: the library reports AHF_ENOMEM
                return None

        def free(user, ptr, nbytes, stream):
            try:
                raw_delete(int(ptr))
            except Exception:
                pass
        # the ctypes thunks must live as long as the context
        self.alloc = ALLOC_FN(alloc)
        self.free = FREE_FN(free)


_lib = None
_hip = None


def load():
    """Load libahf.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: the HIP library must be built first")
    # torch ships its own HIP runtime; loading it first makes libahf.so bind to
    # that same runtime (matched by soname) instead of a second copy
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.ahf_last_error.restype = C.c_char_p
    L.ahf_ctx_create.argtypes = [C.POINTER(CtxDesc), C.POINTER(vp)]
    L.ahf_ctx_destroy.argtypes = [vp]
    L.ahf_ctx_destroy.restype = None
    L.ahf_build_hierarchy.argtypes = [vp, C.POINTER(Particles), C.POINTER(Params), vp, C.POINTER(vp)]
    L.ahf_label_refinements.argtypes = [vp, vp, vp]
    L.ahf_hierarchy_num_levels.argtypes = [vp, C.POINTER(C.c_uint32)]
    L.ahf_level_get.argtypes = [vp, C.c_uint32, C.POINTER(LevelView)]
    L.ahf_hierarchy_order.argtypes = [vp, C.POINTER(vp)]
    L.ahf_hierarchy_timings.argtypes = [vp, C.POINTER(C.c_double), C.c_uint32]
    L.ahf_ctx_set_profiling.argtypes = [vp, C.c_int]
    L.ahf_ctx_kernel_time.argtypes = [vp, C.c_char_p, C.POINTER(C.c_uint64), C.POINTER(C.c_double)]
    L.ahf_ctx_profile_only.argtypes = [vp, C.c_char_p]
    L.ahf_ctx_set_tuning.argtypes = [vp, C.c_uint32, vp, C.POINTER(Tuning)]
    L.ahf_ctx_get_tuning.argtypes = [vp, C.c_uint64, C.POINTER(Tuning)]
    L.ahf_ctx_set_planning.argtypes = [vp, C.c_int]
    L.ahf_hierarchy_build_info.argtypes = [vp, C.POINTER(BuildInfo)]
    L.ahf_classify_substructure.argtypes = [vp, vp, vp]
    L.ahf_hierarchy_structures.argtypes = [vp, C.POINTER(Structures)]
    L.ahf_hierarchy_free.argtypes = [vp]
    L.ahf_hierarchy_free.restype = None
    L.ahf_hierarchy_query_label.argtypes = [vp, vp, C.c_uint32, C.c_uint64, vp, vp, vp]
    L.ahf_hierarchy_query_label_static.argtypes = [vp, C.c_uint32, C.c_uint64, vp, vp, vp]
    L.ahf_server_create.argtypes = [vp, C.POINTER(ServerDesc), C.POINTER(vp)]
    L.ahf_submit.argtypes = [vp, C.POINTER(Particles), C.POINTER(Params), C.POINTER(C.c_uint64)]
    L.ahf_poll.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
    L.ahf_wait.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
    L.ahf_query_label.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint64, vp, vp]
    L.ahf_release.argtypes = [vp, C.c_uint64]
    L.ahf_ticket_times.argtypes = [vp, C.c_uint64, C.POINTER(C.c_double)]
    L.ahf_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    L.ahf_server_destroy.argtypes = [vp]
    L.ahf_server_destroy.restype = None
    L.ahf_batch_create.argtypes = [vp, C.c_uint32, C.POINTER(Particles), C.POINTER(Params),
                                   C.c_uint32, C.c_uint32, vp, C.POINTER(vp)]
    L.ahf_batch_run.argtypes = [vp, vp]
    L.ahf_batch_wait.argtypes = [vp]
    L.ahf_batch_status.argtypes = [vp, C.c_uint32]
    L.ahf_batch_hierarchy.argtypes = [vp, C.c_uint32, C.POINTER(vp)]
    L.ahf_batch_destroy.argtypes = [vp]
    L.ahf_batch_destroy.restype = None
    L.ahf_find_halos.argtypes = [vp, vp, C.POINTER(Particles), vp, vp, vp,
                                 C.POINTER(HaloParams), vp, C.POINTER(vp)]
    L.ahf_halos_get.argtypes = [vp, C.POINTER(HalosView)]
    L.ahf_halos_free.argtypes = [vp]
    L.ahf_halos_free.restype = None
    for name in EXPORTS:
        if name not in ("ahf_ctx_destroy", "ahf_hierarchy_free", "ahf_last_error",
                        "ahf_server_destroy", "ahf_batch_destroy", "ahf_halos_free"):
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def _hip_runtime():
    """libamdhip64 for device-to-host copies of the level arrays."""
    global _hip
    if _hip is None:
        load()  # the runtime already in the process, found by its soname
        for name in ("libamdhip64.so.7", "libamdhip64.so"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("libamdhip64.so not found")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip


def to_host(ptr: int | None, n: int, dtype) -> np.ndarray | None:
    """Copy n elements at device address ptr into a new numpy array."""
    if not ptr:
        return None
    out = np.empty(int(n), dtype=dtype)
    if n:
        rc = _hip_runtime().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed with {rc}")
    return out


def _check(rc):
    if rc != AHF_OK:
        msg = load().ahf_last_error()
        raise AhfError(rc, msg.decode() if msg else "")


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Context:
    """A library context.  memory="torch" (default): device memory comes from
    PyTorch's caching allocator through ahf_ctx_desc's callbacks; "pool": the
    library's own caching pool on hipMalloc; or any object with ctypes
    callbacks `alloc` (ALLOC_FN) and `free` (FREE_FN)."""

    def __init__(self, device: int = 0, memory="torch", tuning="auto"):
        L = load()
        if memory == "torch":
            memory = TorchMemory()
        elif memory == "pool":
            memory = None
        self._memory = memory  # keeps the callbacks alive
        if memory is None:
            d = CtxDesc(C.sizeof(CtxDesc), int(device), None, None, None)
        else:
            d = CtxDesc(C.sizeof(CtxDesc), int(device), C.cast(memory.alloc, C.c_void_p),
                        C.cast(memory.free, C.c_void_p), None)
        h = C.c_void_p()
        _check(L.ahf_ctx_create(C.byref(d), C.byref(h)))
        self._h = h
        self.device = device
        self._live = weakref.WeakSet()  # hierarchies drawing on this context's memory
        # tuning="auto": the autotuner's table for this GPU, if it has been
        # made (paper_0904_3662_amd/autotune.py); None: the library defaults;
        # or a table [(min_n, dict)]
        if tuning == "auto":
            from paper_0904_3662_amd import autotune
            tuning = autotune.load_table()
        if tuning:
            self.set_tuning(tuning)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            for h in list(self._live):
                h.free()
            load().ahf_ctx_destroy(self._h)
            self._h = None

    def set_profiling(self, on: bool):
        _check(load().ahf_ctx_set_profiling(self._h, 1 if on else 0))

    def profile_only(self, names):
        """Time only these kernel names (a list; None or [] = all)."""
        _check(load().ahf_ctx_profile_only(self._h, ",".join(names or []).encode()))

    def set_tuning(self, table):
        """table: list of (min_n, dict(heavy_level0=, heavy_level1=,
        heavy_deeper=, batch_level1=[, sort_skip_digits=])); a build of n
        particles uses the entry with the largest min_n <= n.  [] restores the
        defaults."""
        n = len(table)
        mins = np.array([int(t[0]) for t in table], np.uint64)
        arr = (Tuning * max(n, 1))()
        for i, (_, d) in enumerate(table):
            arr[i] = Tuning(C.sizeof(Tuning), int(d["heavy_level0"]), int(d["heavy_level1"]),
                            int(d["heavy_deeper"]), int(d["batch_level1"]),
                            int(d.get("sort_skip_digits", -1)))
        _check(load().ahf_ctx_set_tuning(self._h, n, mins.ctypes.data if n else None, arr))

    def set_planning(self, on: bool):
        """Builds sized ahead from what earlier builds of the same class
        needed, with no host wait per level (off by default); off also
        forgets the plans."""
        _check(load().ahf_ctx_set_planning(self._h, 1 if on else 0))

    def tuning(self, n: int) -> dict:
        t = Tuning()
        _check(load().ahf_ctx_get_tuning(self._h, int(n), C.byref(t)))
        return {k: int(getattr(t, k)) for k, _ in Tuning._fields_ if k != "struct_size"}

    def kernel_time(self, name: str):
        """(launches, total device ms) of one kernel while profiling."""
        n = C.c_uint64()
        t = C.c_double()
        _check(load().ahf_ctx_kernel_time(self._h, name.encode(), C.byref(n), C.byref(t)))
        return int(n.value), float(t.value)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def make_params(g, dom_ref, ref_ref, max_levels, connectivity=26, flags=0) -> Params:
    return Params(C.sizeof(Params), int(g), float(dom_ref), float(ref_ref), int(max_levels),
                  int(connectivity), int(flags))


def make_particles(x, y, z, fx=None, fy=None, fz=None, mass=None, mass_scalar=1.0) -> Particles:
    for t in (x, y, z):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("x, y, z must be contiguous device tensors")
    return Particles(int(x.numel()), _ptr(x), _ptr(y), _ptr(z), _ptr(fx), _ptr(fy), _ptr(fz),
                     _ptr(mass), float(mass_scalar))


class Hierarchy:
    """A built hierarchy; level arrays stay on the device until copied."""

    def __init__(self, handle, ctx=None, keep=None, borrowed=False):
        self._h = handle
        self._ctx = ctx
        self._keep = keep  # input tensors stay alive while the build may read them
        self._borrowed = borrowed  # owned by a server: never freed from here
        if ctx is not None and not borrowed:
            ctx._live.add(self)

    @property
    def handle(self):
        return self._h

    def num_levels(self) -> int:
        n = C.c_uint32()
        _check(load().ahf_hierarchy_num_levels(self._h, C.byref(n)))
        return int(n.value)

    def view(self, level: int) -> LevelView:
        v = LevelView()
        _check(load().ahf_level_get(self._h, int(level), C.byref(v)))
        return v

    def order_ptr(self) -> int:
        p = C.c_void_p()
        _check(load().ahf_hierarchy_order(self._h, C.byref(p)))
        return p.value or 0

    def build_info(self) -> dict:
        b = BuildInfo()
        _check(load().ahf_hierarchy_build_info(self._h, C.byref(b)))
        return {k: int(getattr(b, k)) for k, _ in BuildInfo._fields_ if k != "struct_size"}

    def timings(self):
        a = (C.c_double * 4)()
        _check(load().ahf_hierarchy_timings(self._h, a, 4))
        return list(a)

    def order_numpy(self, n: int) -> np.ndarray:
        out = to_host(self.order_ptr(), n, np.uint32)
        return np.zeros(0, np.uint32) if out is None else out

    def level_numpy(self, level: int) -> dict:
        v = self.view(level)
        nS, nB, nP = v.n_cells, v.n_bricks, v.n_patches
        d = dict(level=v.level, bits=v.bits, n_cells=nS, n_refined=v.n_refined,
                 n_particles=v.n_particles, n_bricks=nB, n_patches=nP,
                 total_cell_mass=v.total_cell_mass,
                 total_particle_mass=v.total_particle_mass)
        d["cell_key"] = to_host(v.cell_key, nS, np.uint64)
        if d["cell_key"] is None:
            d["cell_key"] = np.arange(nS, dtype=np.uint64)
        d["cell_start"] = to_host(v.cell_start, nS, np.uint32)
        d["cell_count"] = to_host(v.cell_count, nS, np.uint32)
        d["cell_refined"] = to_host(v.cell_refined, nS, np.uint8)
        d["cell_patch"] = to_host(v.cell_patch, nS, np.int32)
        bk = to_host(v.brick_key, nB, np.uint64)
        d["brick_key"] = np.arange(nB, dtype=np.uint64) if bk is None else bk
        bc = to_host(v.brick_cell, nB, np.int32)
        d["brick_cell"] = (np.arange(nB, dtype=np.int64) * 8).astype(np.int32) if bc is None else bc
        d["brick_mass"] = to_host(v.brick_mass, 8 * nB, np.float32)
        d["patch_parent"] = to_host(v.patch_parent, nP, np.int32)
        d["patch_ncells"] = to_host(v.patch_ncells, nP, np.uint32)
        d["patch_nparticles"] = to_host(v.patch_nparticles, nP, np.uint64)
        d["patch_mass"] = to_host(v.patch_mass, nP, np.float64)
        d["patch_struct"] = to_host(v.patch_struct, nP, np.int32)
        return d

    def classify(self, ctx: "Context", stream=None):
        """Host structures and substructures of the (labelled) grid tree."""
        _check(load().ahf_classify_substructure(ctx.handle, self._h, _stream_handle(stream)))

    def structures(self) -> dict:
        s = Structures()
        _check(load().ahf_hierarchy_structures(self._h, C.byref(s)))
        n = s.n_structures
        out = {"n_structures": n}
        for k in ("host", "level", "patch", "depth"):
            a = to_host(getattr(s, k), n, np.int32)
            out[k] = np.zeros(0, np.int32) if a is None else a
        return out

    def label(self, ctx: Context, stream=None):
        _check(load().ahf_label_refinements(ctx.handle, self._h, _stream_handle(stream)))

    def query_label(self, ctx: "Context", level: int, keys: np.ndarray, stream=None) -> np.ndarray:
        """Patch id of each level cell given by key (-1 outside S_L)."""
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(len(k), np.int32)
        _check(load().ahf_hierarchy_query_label(ctx.handle, self._h, int(level), len(k),
                                                k.ctypes.data, out.ctypes.data,
                                                _stream_handle(stream)))
        return out

    def query_label_static(self, level: int, keys: np.ndarray, stream=None) -> np.ndarray:
        """query_label through the library's static staging area (allocates
        no device memory; at most 262144 keys per call)."""
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(len(k), np.int32)
        _check(load().ahf_hierarchy_query_label_static(self._h, int(level), len(k),
                                                       k.ctypes.data, out.ctypes.data,
                                                       _stream_handle(stream)))
        return out

    def free(self):
        if self._h:
            if not self._borrowed and (self._ctx is None or self._ctx._h):
                load().ahf_hierarchy_free(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        # at interpreter exit the allocator behind the context may be gone
        # (and this module's globals may already be cleared)
        if sys is None or sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def build_hierarchy(ctx: Context, x, y, z, fx=None, fy=None, fz=None, mass=None, *,
                    g: int, dom_ref: float, ref_ref: float, max_levels: int,
                    connectivity: int = 26, labels: bool = True, mass_scalar: float = 1.0,
                    substructure: bool = False, density_criterion: bool = False,
                    stream=None) -> Hierarchy:
    parts = make_particles(x, y, z, fx, fy, fz, mass, mass_scalar)
    prm = make_params(g, dom_ref, ref_ref, max_levels, connectivity,
                      _flags(labels, substructure, density_criterion))
    h = C.c_void_p()
    _check(load().ahf_build_hierarchy(ctx.handle, C.byref(parts), C.byref(prm),
                                      _stream_handle(stream), C.byref(h)))
    return Hierarchy(h, ctx=ctx, keep=(x, y, z, fx, fy, fz, mass))


def snapshot_to_device(s, device="cuda"):
    """numpy snapshot arrays -> device tensors (x, y, z, fx, fy, fz, mass or None)."""
    import torch
    def t(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
    # uint32 coordinates travel as int32 bit patterns (torch has no uint32 kernels)
    X = t(s.X.view(np.int32)); Y = t(s.Y.view(np.int32)); Z = t(s.Z.view(np.int32))
    return X, Y, Z, t(s.fx), t(s.fy), t(s.fz), t(s.mass)


def build_snapshot(ctx: Context, s, labels=True, connectivity=26, stream=None, dev=None,
                   substructure=False, density_criterion=False):
    """Build the hierarchy of a synth.Snapshot (copies it to the device first
    unless `dev` already holds its device tensors)."""
    dev = dev if dev is not None else snapshot_to_device(s)
    return build_hierarchy(ctx, *dev[:6], dev[6], g=s.g, dom_ref=s.dom_ref, ref_ref=s.ref_ref,
                           max_levels=s.max_levels, connectivity=connectivity, labels=labels,
                           substructure=substructure, density_criterion=density_criterion,
                           stream=stream), dev


def _flags(labels, substructure, density_criterion=False):
    return ((0 if labels else AHF_NO_LABELS) | (AHF_SUBSTRUCTURE if substructure else 0)
            | (AHF_DENSITY_CRITERION if density_criterion else 0))


class Server:
    """Continuous-batching server (ahf_server_*): requests overlap on the GPU."""

    def __init__(self, ctx: Context, n_streams: int = 4, max_queue: int = 0,
                 hbm_budget: int = 0):
        d = ServerDesc(C.sizeof(ServerDesc), int(n_streams), int(max_queue), 0, int(hbm_budget))
        h = C.c_void_p()
        _check(load().ahf_server_create(ctx.handle, C.byref(d), C.byref(h)))
        self._h = h
        self._ctx = ctx
        self._inputs = {}  # ticket -> tensors the build reads

    def submit(self, x, y, z, fx=None, fy=None, fz=None, mass=None, *, g, dom_ref, ref_ref,
               max_levels, connectivity=26, labels=True, mass_scalar=1.0,
               substructure=False) -> int:
        parts = make_particles(x, y, z, fx, fy, fz, mass, mass_scalar)
        prm = make_params(g, dom_ref, ref_ref, max_levels, connectivity,
                          _flags(labels, substructure))
        t = C.c_uint64()
        _check(load().ahf_submit(self._h, C.byref(parts), C.byref(prm), C.byref(t)))
        self._inputs[t.value] = (x, y, z, fx, fy, fz, mass)
        return int(t.value)

    def submit_snapshot(self, snap, dev=None, connectivity=26, labels=True,
                        substructure=False) -> int:
        dev = dev if dev is not None else snapshot_to_device(snap)
        return self.submit(*dev[:6], dev[6], g=snap.g, dom_ref=snap.dom_ref,
                           ref_ref=snap.ref_ref, max_levels=snap.max_levels,
                           connectivity=connectivity, labels=labels, substructure=substructure)

    def _result(self, rc, ticket, h):
        if rc == AHF_PENDING:
            return None
        self._inputs.pop(ticket, None)
        _check(rc)
        return Hierarchy(h, borrowed=True)

    def poll(self, ticket: int):
        """None while pending, else the (borrowed) Hierarchy; raises on failure."""
        h = C.c_void_p()
        return self._result(load().ahf_poll(self._h, C.c_uint64(ticket), C.byref(h)), ticket, h)

    def wait(self, ticket: int):
        h = C.c_void_p()
        return self._result(load().ahf_wait(self._h, C.c_uint64(ticket), C.byref(h)), ticket, h)

    def query_label(self, ticket: int, level: int, keys: np.ndarray) -> np.ndarray:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(len(k), np.int32)
        _check(load().ahf_query_label(self._h, C.c_uint64(ticket), int(level), len(k),
                                      k.ctypes.data, out.ctypes.data))
        return out

    def release(self, ticket: int):
        _check(load().ahf_release(self._h, C.c_uint64(ticket)))

    def times(self, ticket: int):
        a = (C.c_double * 4)()
        _check(load().ahf_ticket_times(self._h, C.c_uint64(ticket), a))
        return list(a)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().ahf_server_get_stats(self._h, C.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            load().ahf_server_destroy(self._h)
            self._h = None
            self._inputs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


AHF_BATCH_GRAPH = 1


class Batch:
    """Sub-volumes rebuilt together, one host wait per run (ahf_batch_*).
    The particle tensors are held for the life of the batch; a run rebuilds
    every sub-volume from their current contents."""

    def __init__(self, ctx: Context, snaps, devs=None, n_chains: int = 4, connectivity=26,
                 labels=True, stream=None, graph: bool = False):
        devs = devs if devs is not None else [snapshot_to_device(s) for s in snaps]
        n = len(snaps)
        parts = (Particles * n)()
        prms = (Params * n)()
        for i, (s, d) in enumerate(zip(snaps, devs)):
            parts[i] = make_particles(*d[:6], d[6])
            prms[i] = make_params(s.g, s.dom_ref, s.ref_ref, s.max_levels, connectivity,
                                  _flags(labels, False))
        h = C.c_void_p()
        _check(load().ahf_batch_create(ctx.handle, n, parts, prms, int(n_chains),
                                       AHF_BATCH_GRAPH if graph else 0,
                                       _stream_handle(stream), C.byref(h)))
        self._h = h
        self._ctx = ctx
        self._keep = devs
        self.n = n

    def run(self, stream=None):
        _check(load().ahf_batch_run(self._h, _stream_handle(stream)))

    def wait(self):
        _check(load().ahf_batch_wait(self._h))

    def status(self, i: int) -> int:
        return int(load().ahf_batch_status(self._h, int(i)))

    def hierarchy(self, i: int) -> Hierarchy:
        h = C.c_void_p()
        _check(load().ahf_batch_hierarchy(self._h, int(i), C.byref(h)))
        return Hierarchy(h, borrowed=True)

    def close(self):
        if self._h:
            load().ahf_batch_destroy(self._h)
            self._h = None
            self._keep = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def find_halos(ctx: Context, h: Hierarchy, dev, vel, delta_vir: float = 340.0, G: float = 1.0,
               max_iter: int = 1000, stream=None, fetch: bool = True,
               large_from: int = 0) -> dict:
    """Particle collection and unbinding of every structure of a classified
    hierarchy (ahf_find_halos); dev holds the particle tensors the hierarchy
    was built from, vel the (n, 3) velocities on the device.  Returns the
    halos as numpy arrays (the device result is freed); without fetch only
    the per-halo counts and rounds."""
    vel = vel.contiguous()
    vx, vy, vz = (vel[:, k].contiguous() for k in range(3))
    parts = make_particles(*dev[:6], dev[6])
    prm = HaloParams(C.sizeof(HaloParams), float(delta_vir), float(G), int(max_iter),
                     int(large_from))
    out = C.c_void_p()
    _check(load().ahf_find_halos(ctx.handle, h.handle, C.byref(parts), _ptr(vx), _ptr(vy),
                                 _ptr(vz), C.byref(prm), _stream_handle(stream), C.byref(out)))
    try:
        v = HalosView()
        _check(load().ahf_halos_get(out, C.byref(v)))
        n = int(v.n_halos)
        res = {"n_halos": n}
        if not fetch:
            res["cand_count"] = to_host(v.cand_count, n, np.uint32)
            res["member_count"] = to_host(v.member_count, n, np.uint32)
            res["iterations"] = to_host(v.iterations, n, np.uint32)
            return res
        res["leaf"] = to_host(v.leaf, n, np.uint64)
        res["centre"] = to_host(v.centre, 3 * n, np.float64).reshape(n, 3)
        res["radius"] = to_host(v.radius, n, np.float64)
        off = to_host(v.cand_offset, n + 1, np.uint64)
        res["cand_offset"] = off
        total = int(off[-1]) if n else 0
        res["cand_count"] = to_host(v.cand_count, n, np.uint32)
        res["member_count"] = to_host(v.member_count, n, np.uint32)
        cand = to_host(v.cand, max(total, 1), np.uint32)
        mem = to_host(v.member, max(total, 1), np.uint32)
        res["candidates"] = [cand[int(off[s]):int(off[s]) + int(res["cand_count"][s])]
                             for s in range(n)]
        res["members"] = [mem[int(off[s]):int(off[s]) + int(res["member_count"][s])]
                          for s in range(n)]
        res["r_vir"] = to_host(v.r_vir, n, np.float64)
        res["m_vir"] = to_host(v.m_vir, n, np.float64)
        res["vel"] = to_host(v.vel, 3 * n, np.float64).reshape(n, 3)
        res["iterations"] = to_host(v.iterations, n, np.uint32)
        return res
    finally:
        load().ahf_halos_free(out)
