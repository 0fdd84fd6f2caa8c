"""ctypes binding of libsss.so (include/sss.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libsss.so.  Tensors must be CUDA (ROCm) tensors on the current
device; work is enqueued on torch's current stream unless a stream is given.
Importing this module loads the library and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsss.so")

TILE = 16
MAX_VIEWS = 16
RECORD_BYTES = 64
ENTRY_BYTES = 128
G2_SLOTS = 12
OK, ERR_INVALID, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED = 0, -1, -2, -3, -4
BWD_STORED, BWD_RECOMPUTE, BWD_DETERMINISTIC = 0, 1, 4
LOSS_GRAD, LOSS_L1 = 0, 1

c_f32p = ctypes.c_void_p


class Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("nu", ctypes.c_void_p), ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class Grads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("nu", ctypes.c_void_p), ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("overwrite", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("viewmat", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float),
                ("z_near", ctypes.c_float), ("nu_min", ctypes.c_float), ("nu_max", ctypes.c_float),
                ("lowpass", ctypes.c_float), ("bg", ctypes.c_float * 3), ("family", ctypes.c_int32),
                ("trunc_mode", ctypes.c_int32)]


class Proj(ctypes.Structure):
    _fields_ = [("entries", ctypes.c_void_p), ("depth_key", ctypes.c_void_p), ("tiles_touched", ctypes.c_void_p)]


class Bins(ctypes.Structure):
    _fields_ = [("order", ctypes.c_void_p), ("sorted_records", ctypes.c_void_p), ("tile_start", ctypes.c_void_p),
                ("pair_rank", ctypes.c_void_p), ("rank_offset", ctypes.c_void_p), ("tile_order", ctypes.c_void_p),
                ("tile_work", ctypes.c_void_p), ("pair_capacity", ctypes.c_int64),
                ("n_visible", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("counts", ctypes.c_void_p),
                ("no_wait", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SghmcOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("friction", ctypes.c_float), ("k", ctypes.c_float), ("t", ctypes.c_float),
                ("burn_in", ctypes.c_int32), ("noise", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("step", ctypes.c_uint64)]


class AdamArray(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("count", ctypes.c_int64), ("lr", ctypes.c_float), ("lo", ctypes.c_float),
                ("hi", ctypes.c_float)]


class Adam(ctypes.Structure):
    _fields_ = [("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("n_arrays", ctypes.c_int32), ("t", ctypes.c_int64), ("arrays", AdamArray * 6)]


class Step(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p * 6), ("momentum", ctypes.c_void_p), ("sghmc", SghmcOpts),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("adam", ctypes.c_int32),
                ("t", ctypes.c_int64), ("m", ctypes.c_void_p * 5), ("v", ctypes.c_void_p * 5),
                ("lr", ctypes.c_float * 5), ("lo", ctypes.c_float * 5), ("hi", ctypes.c_float * 5)]


class RelocateOpts(ctypes.Structure):
    _fields_ = [("dead_opacity", ctypes.c_float), ("max_fraction", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("step", ctypes.c_uint64)]


class StateArray(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("width", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


# every function include/sss.h declares; lib() checks that each is exported
EXPORTS = ["sss_default_render_opts", "sss_project", "sss_bin_sort", "sss_bin_sort_workspace", "sss_total_tiles",
           "sss_total_pixels", "sss_render_fwd", "sss_render_bwd", "sss_render_bwd_workspace",
           "sss_render_bwd_workspace_det", "sss_render_bwd_noalloc", "sss_render_bwd_step", "sss_sghmc_step",
           "sss_loss",
           "sss_loss_workspace", "sss_regularise", "sss_relocate", "sss_relocate_workspace", "sss_timing_enable",
           "sss_timing_reset", "sss_timing_read", "sss_stream_copy", "sss_last_error", "sss_version"]

_lib = None


def lib():
    """Load libsss.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_10148_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        missing = [name for name in EXPORTS if not hasattr(L, name)]
        if missing:
            raise RuntimeError(f"{LIB_PATH} does not export {missing}: rebuild it")
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.sss_last_error.restype = ctypes.c_char_p
        L.sss_version.restype = i32
        L.sss_bin_sort_workspace.restype = ctypes.c_size_t
        L.sss_bin_sort_workspace.argtypes = [i64, i64]
        L.sss_render_bwd_workspace.restype = ctypes.c_size_t
        L.sss_render_bwd_workspace.argtypes = [i64, i64]
        L.sss_render_bwd_workspace_det.restype = ctypes.c_size_t
        L.sss_render_bwd_workspace_det.argtypes = [i64, i64, i64]
        L.sss_total_tiles.restype = i64
        L.sss_total_tiles.argtypes = [vp, i32]
        L.sss_total_pixels.restype = i64
        L.sss_total_pixels.argtypes = [vp, i32]
        L.sss_project.argtypes = [vp, vp, i32, vp, vp, vp]
        L.sss_bin_sort.argtypes = [vp, vp, i32, i64, vp, vp, ctypes.c_size_t, vp]
        L.sss_render_fwd.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
        L.sss_render_bwd.argtypes = [vp, vp, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp,
                                     ctypes.c_size_t, vp]
        L.sss_render_bwd_noalloc.argtypes = [vp, vp, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.sss_render_bwd_step.argtypes = [vp, vp, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                          ctypes.c_size_t, vp]
        L.sss_sghmc_step.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp]
        L.sss_loss_workspace.restype = ctypes.c_size_t
        L.sss_loss_workspace.argtypes = [i64]
        L.sss_loss.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, ctypes.c_size_t, vp]
        L.sss_loss.restype = i32
        L.sss_regularise.argtypes = [vp, vp, i64, ctypes.c_float, ctypes.c_float, vp, vp, vp, vp]
        L.sss_regularise.restype = i32
        L.sss_relocate_workspace.restype = ctypes.c_size_t
        L.sss_relocate_workspace.argtypes = [i64, ctypes.c_float]
        L.sss_relocate.argtypes = [vp, vp, i32, vp, vp, ctypes.c_size_t, vp, vp]
        L.sss_relocate.restype = i32
        L.sss_timing_enable.argtypes = [i32]
        L.sss_timing_enable.restype = i32
        L.sss_timing_reset.restype = None
        L.sss_timing_read.argtypes = [vp, i32]
        L.sss_timing_read.restype = i32
        L.sss_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.sss_stream_copy.restype = i32
        for name in ("sss_project", "sss_bin_sort", "sss_render_fwd", "sss_render_bwd", "sss_render_bwd_noalloc",
                     "sss_render_bwd_step", "sss_sghmc_step"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


class SSSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _check(rc, what):
    if rc != OK:
        raise SSSError(rc, f"{what}: {lib().sss_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _addr(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


# ---------------------------------------------------------------------------
# argument structs
# ---------------------------------------------------------------------------
class CameraBatch:
    """Cameras marshalled once into the C-ABI's array, with the batch's
    total tiles and pixels.  Every call that takes `cams` accepts either a
    list of camera dicts or a CameraBatch (reuse it across the calls of one
    step or one request to skip repeated marshalling)."""

    def __init__(self, cams):
        cams = list(cams)
        self.cams = cams
        self.array = (Camera * len(cams))()
        for i, c in enumerate(cams):
            vm = c["viewmat"]
            vm = vm.reshape(-1).tolist() if hasattr(vm, "reshape") else [x for row in vm for x in row]
            self.array[i].viewmat[:] = [float(x) for x in vm]
            self.array[i].fx, self.array[i].fy, self.array[i].cx, self.array[i].cy = c["fx"], c["fy"], c["cx"], c["cy"]
            self.array[i].width, self.array[i].height = int(c["width"]), int(c["height"])
        self.n_tiles = int(lib().sss_total_tiles(self.array, len(cams)))
        self.n_pixels = int(lib().sss_total_pixels(self.array, len(cams)))

    def __len__(self):
        return len(self.cams)

    def __getitem__(self, k):
        return self.cams[k]

    def __iter__(self):
        return iter(self.cams)


def camera_batch(cams) -> CameraBatch:
    return cams if isinstance(cams, CameraBatch) else CameraBatch(cams)


def camera_array(cams):
    return camera_batch(cams).array


def render_opts(opts=None):
    """dict of overrides (or None) -> RenderOpts; a RenderOpts is passed through."""
    if isinstance(opts, RenderOpts):
        return opts
    o = RenderOpts()
    lib().sss_default_render_opts(ctypes.byref(o))
    for k, v in (opts or {}).items():
        if k == "bg":
            o.bg[:] = [float(x) for x in v]
        elif k == "family":
            o.family = {"student_t": 0, "gaussian": 1}.get(v, v) if isinstance(v, str) else int(v)
        elif k == "trunc_mode":
            o.trunc_mode = {"alpha": 0, "coverage": 1}.get(v, v) if isinstance(v, str) else int(v)
        else:
            setattr(o, k, float(v))
    return o


def scene_struct(scene):
    """scene: dict of CUDA float32 tensors means [n,3], scales [n,3], quats [n,4],
    nu [n], opacity [n], sh [n,K,3] and an int sh_degree."""
    n = scene["means"].shape[0]
    for k in ("means", "scales", "quats", "nu", "opacity", "sh"):
        _need(scene[k], torch.float32, k)
    return Scene(n, int(scene["sh_degree"]), 0, *(scene[k].data_ptr() for k in
                                                   ("means", "scales", "quats", "nu", "opacity", "sh")))


def scene_to_device(scene, device="cuda"):
    """numpy scene dict -> dict of contiguous float32 tensors on `device`."""
    import numpy as np
    out = {k: torch.as_tensor(np.ascontiguousarray(scene[k]), dtype=torch.float32, device=device)
           for k in ("means", "scales", "quats", "nu", "opacity", "sh")}
    out["sh_degree"] = int(scene["sh_degree"])
    return out


def total_tiles(cams):
    return camera_batch(cams).n_tiles


def total_pixels(cams):
    return camera_batch(cams).n_pixels


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------
@dataclass
class Projected:
    entries: torch.Tensor      # uint8 [E, 128]: record, FP64 ellipse, tile rectangle (include/sss.h)
    depth_key: torch.Tensor    # int32 [E] (uint32 bits)
    touched: torch.Tensor      # int32 [E]

    @property
    def records(self) -> torch.Tensor:
        """uint8 [E, 64] view: the raster records."""
        return self.entries[:, :RECORD_BYTES]

    @property
    def ellipse(self) -> torch.Tensor:
        """float64 [E, 4] view: 2D covariance A, B, D and the listed level."""
        return self.entries[:, 64:96].view(torch.float64)

    @property
    def rect(self) -> torch.Tensor:
        """int16 [E, 4] view: tile rectangle x0, y0, x1, y1 (uint16 bits)."""
        return self.entries[:, 96:104].view(torch.int16)

    def struct(self):
        return Proj(self.entries.data_ptr(), self.depth_key.data_ptr(), self.touched.data_ptr())


def project(scene, cams, opts=None, stream=None, out: Projected | None = None) -> Projected:
    cams = camera_batch(cams)
    n = scene["means"].shape[0]
    E = n * len(cams)
    dev = scene["means"].device
    if out is None:
        out = Projected(torch.empty((E, ENTRY_BYTES), dtype=torch.uint8, device=dev),
                        torch.empty(E, dtype=torch.int32, device=dev),
                        torch.empty(E, dtype=torch.int32, device=dev))
    s = scene_struct(scene)
    p = out.struct()
    _check(lib().sss_project(ctypes.byref(s), cams.array, len(cams), ctypes.byref(render_opts(opts)),
                             ctypes.byref(p), _stream(stream)), "sss_project")
    return out


@dataclass
class Binned:
    order: torch.Tensor          # int32 [E]
    sorted_records: torch.Tensor # uint8 [E, 64]
    tile_start: torch.Tensor     # int32 [tiles + 1]
    pair_rank: torch.Tensor      # int32 [capacity]
    n_visible: int = 0
    n_pairs: int = 0
    rank_offset: torch.Tensor | None = None   # int32 [E], kept for the deterministic backward
    tile_order: torch.Tensor | None = None    # int32 [tiles], launch order (longest list first)
    tile_work: torch.Tensor | None = None     # int32 [tiles, 4], per 16x4 strip the largest n_contrib (render_fwd)
    counts: torch.Tensor | None = None        # int64 [2] device: visible entries, required pairs (no-wait calls)
    capacity: int = 0                         # pairs the call could hold (0: all of pair_rank)

    def cap(self) -> int:
        return self.capacity if self.capacity > 0 else self.pair_rank.numel()

    def struct(self, no_wait: bool = False):
        return Bins(self.order.data_ptr(), self.sorted_records.data_ptr(), self.tile_start.data_ptr(),
                    self.pair_rank.data_ptr(), _addr(self.rank_offset), _addr(self.tile_order),
                    _addr(self.tile_work), self.cap(), self.n_visible, self.n_pairs,
                    _addr(self.counts), int(no_wait), 0)

    def resolve(self):
        """After a no-wait binning: wait for its counts, fill n_visible and
        n_pairs, and raise SSSError(ERR_CAPACITY) if the lists were cut short
        by the pair capacity."""
        if self.n_pairs < 0:
            c = self.counts.cpu()
            self.n_visible, self.n_pairs = int(c[0]), int(c[1])
        if self.n_pairs > self.cap():
            raise SSSError(ERR_CAPACITY, f"sss_bin_sort: {self.n_pairs} pairs exceed the capacity {self.cap()}")
        return self


class BinSorter:
    """Holds the pair and workspace buffers of sss_bin_sort and grows them
    (with 25% headroom) when a call reports SSS_ERR_CAPACITY.  With
    `schedule` (default), the Binned it creates carries the tile launch
    order and per-tile work arrays, so the raster kernels start the most
    expensive tiles first.

    By default every Binned the sorter returns shares the sorter's one pair
    list (the next call overwrites it), which suits a loop that consumes
    each binning before the next.  With `own_pairs`, each call gets a pair
    list of its own, so several binnings can be alive at once (renders
    whose backward passes run later).

    With `no_wait`, calls after the first never wait for the device: the
    counts go to a device tensor (`counts`, or one the sorter keeps) and
    the returned Binned has n_visible = n_pairs = -1 until `resolve()`; a
    binning whose pairs exceeded the capacity must be redone (resolve()
    raises, and the sorter grows its capacity for the next call).  The
    first call, with no capacity yet, waits to size the buffers."""

    def __init__(self, pair_capacity: int = 0, keep_offsets: bool = False, schedule: bool = True,
                 own_pairs: bool = False, no_wait: bool = False, headroom: float = 1.25, work: bool = True):
        self.cap = int(pair_capacity)
        self.ws = None
        self.pair_rank = None
        self.keep_offsets = keep_offsets
        self.schedule = schedule
        self.own_pairs = own_pairs
        self.no_wait = no_wait
        self.headroom = float(headroom)
        self.work = work           # per-strip walk lengths for a later backward pass
        self.counts = None

    def grow(self, n_pairs: int):
        """Make the next calls' capacity hold n_pairs with the headroom."""
        self.cap = max(self.cap, int(n_pairs * self.headroom) + 1024)

    def __call__(self, proj: Projected, cams, n: int, stream=None, out: Binned | None = None,
                 counts: torch.Tensor | None = None, capacity: int | None = None) -> Binned:
        """capacity (no-wait calls): the most pairs this call may emit, if
        less than the pair buffer holds; the pair passes' grids are sized by
        it, so a good estimate keeps small calls cheap on large buffers (a
        call that needs more must be redone: resolve() raises)."""
        cams = camera_batch(cams)
        E = n * len(cams)
        dev = proj.entries.device
        T = total_tiles(cams)
        if out is None:
            out = Binned(torch.empty(E, dtype=torch.int32, device=dev),
                         torch.empty((E, RECORD_BYTES), dtype=torch.uint8, device=dev),
                         torch.empty(T + 1, dtype=torch.int32, device=dev), None)
            if self.schedule:
                out.tile_order = torch.empty(T, dtype=torch.int32, device=dev)
                if self.work:
                    out.tile_work = torch.empty((T, 4), dtype=torch.int32, device=dev)
        if self.keep_offsets and (out.rank_offset is None or out.rank_offset.numel() < E):
            out.rank_offset = torch.empty(E, dtype=torch.int32, device=dev)
        camarr = cams.array
        p = proj.struct()
        no_wait = self.no_wait and self.cap > 0
        if no_wait:
            if counts is None:
                if self.counts is None:
                    self.counts = torch.empty(2, dtype=torch.int64, device=dev)
                counts = self.counts
        out.counts = counts
        pairs = None
        for _ in range(3):
            if self.own_pairs:
                if pairs is None or pairs.numel() < max(self.cap, 1):
                    pairs = torch.empty(max(self.cap, 1), dtype=torch.int32, device=dev)
            else:
                if self.pair_rank is None or self.pair_rank.numel() < max(self.cap, 1):
                    self.pair_rank = torch.empty(max(self.cap, 1), dtype=torch.int32, device=dev)
                pairs = self.pair_rank
            need = int(lib().sss_bin_sort_workspace(E, pairs.numel()))
            if self.ws is None or self.ws.numel() < need:
                self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
            out.pair_rank = pairs
            out.capacity = min(pairs.numel(), max(int(capacity), 1)) if (no_wait and capacity) else 0
            b = out.struct(no_wait)
            rc = lib().sss_bin_sort(ctypes.byref(p), camarr, len(cams), n, ctypes.byref(b), _ptr(self.ws),
                                    self.ws.numel(), _stream(stream))
            out.n_visible, out.n_pairs = int(b.n_visible), int(b.n_pairs)
            if rc == ERR_CAPACITY:
                self.grow(b.n_pairs)
                continue
            _check(rc, "sss_bin_sort")
            return out
        raise SSSError(ERR_CAPACITY, "sss_bin_sort: capacity retry did not converge")


def render_fwd(bins: Binned, cams, opts=None, stream=None, image=None, t_final=None, n_contrib=None, aux=True):
    """aux=False: only the image (no final transmittance, no list positions:
    a render that no backward pass will use)."""
    cams = camera_batch(cams)
    P = cams.n_pixels
    dev = bins.order.device
    image = torch.empty((P, 3), dtype=torch.float32, device=dev) if image is None else image
    if aux:
        t_final = torch.empty(P, dtype=torch.float32, device=dev) if t_final is None else t_final
        n_contrib = torch.empty(P, dtype=torch.int32, device=dev) if n_contrib is None else n_contrib
    b = bins.struct()
    _check(lib().sss_render_fwd(ctypes.byref(b), cams.array, len(cams), ctypes.byref(render_opts(opts)),
                                _ptr(image), _ptr(t_final), _ptr(n_contrib), _stream(stream)), "sss_render_fwd")
    return image, t_final, n_contrib


def zero_grads_like(scene):
    return {k: torch.zeros_like(scene[k]) for k in ("means", "scales", "quats", "nu", "opacity", "sh")}


def render_bwd(scene, proj: Projected, bins: Binned, cams, dl_or_target, opts=None, mode=BWD_STORED,
               loss=LOSS_GRAD, image=None, n_contrib=None, image_out=None, loss_out=None, grads=None,
               ws=None, stream=None, overwrite=None, deterministic=False, noalloc=False):
    """Gradients into `grads` (+= by default; written when overwrite, which is
    the default when grads is None and new buffers are allocated).
    deterministic: no float atomics, bit-identical results run to run (needs
    bins from BinSorter(keep_offsets=True)).
    noalloc: call sss_render_bwd_noalloc, whose workspace the library holds
    (up to SSS_NOALLOC_WORKSPACE_BYTES); `ws` is ignored."""
    cams = camera_batch(cams)
    n = scene["means"].shape[0]
    E = n * len(cams)
    if grads is None:
        grads = {k: torch.empty_like(scene[k]) for k in ("means", "scales", "quats", "nu", "opacity", "sh")}
        overwrite = True if overwrite is None else overwrite
    overwrite = bool(overwrite)
    if deterministic:
        mode |= BWD_DETERMINISTIC
        need = int(lib().sss_render_bwd_workspace_det(E, bins.n_pairs, total_tiles(cams)))
    else:
        need = int(lib().sss_render_bwd_workspace(E, total_tiles(cams)))
    s = scene_struct(scene)
    g = Grads(*(grads[k].data_ptr() for k in ("means", "scales", "quats", "nu", "opacity", "sh")), int(overwrite), 0)
    p = proj.struct()
    b = bins.struct()
    if noalloc:
        _check(lib().sss_render_bwd_noalloc(ctypes.byref(s), ctypes.byref(p), ctypes.byref(b), cams.array,
                                            len(cams), ctypes.byref(render_opts(opts)), mode, loss,
                                            _ptr(dl_or_target), _ptr(image), _ptr(n_contrib), _ptr(image_out),
                                            _ptr(loss_out), ctypes.byref(g), _stream(stream)),
               "sss_render_bwd_noalloc")
        return grads
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need // 4, dtype=torch.float32, device=scene["means"].device)
    _check(lib().sss_render_bwd(ctypes.byref(s), ctypes.byref(p), ctypes.byref(b), cams.array, len(cams),
                                ctypes.byref(render_opts(opts)), mode, loss, _ptr(dl_or_target), _ptr(image),
                                _ptr(n_contrib), _ptr(image_out), _ptr(loss_out), ctypes.byref(g), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)), "sss_render_bwd")
    return grads


def sghmc_step(means, momentum, grad_means, opacity, lr, friction=0.1, k=100.0, t=0.995, burn_in=False,
               noise=True, seed=0, step=0, scales=None, quats=None, adam=None, stream=None):
    """In-place SGHMC step on `means`/`momentum`.  adam: optional dict with
    beta1, beta2, eps, t and a list 'arrays' of dicts (param, grad, m, v, lr, lo, hi)."""
    o = SghmcOpts(lr, friction, k, t, int(burn_in), int(noise), seed, step)
    ad = None
    if adam is not None:
        ad = Adam()
        ad.beta1, ad.beta2, ad.eps = adam.get("beta1", 0.9), adam.get("beta2", 0.999), adam.get("eps", 1e-15)
        ad.t = int(adam["t"])
        ad.n_arrays = len(adam["arrays"])
        for i, a in enumerate(adam["arrays"]):
            ad.arrays[i] = AdamArray(a["param"].data_ptr(), a["grad"].data_ptr(), a["m"].data_ptr(),
                                     a["v"].data_ptr(), a["param"].numel(), a["lr"], a.get("lo", -3.0e38),
                                     a.get("hi", 3.0e38))
    _check(lib().sss_sghmc_step(_ptr(means), _ptr(momentum), _ptr(grad_means), _ptr(opacity), _ptr(scales),
                                _ptr(quats), means.shape[0], ctypes.byref(o),
                                ctypes.byref(ad) if ad is not None else None, _stream(stream)), "sss_sghmc_step")


STEP_ARRAYS = ("scales", "quats", "nu", "opacity", "sh")


def render_bwd_step(scene, proj: Projected, bins: Binned, cams, dl_or_target, momentum, sghmc: dict,
                    adam: dict | None = None, opts=None, mode=BWD_STORED, loss=LOSS_GRAD, image=None, n_contrib=None,
                    image_out=None, loss_out=None, grads=None, ws=None, stream=None, deterministic=False):
    """sss_render_bwd_step: the backward pass with the SGHMC step on the
    means and Adam on the other arrays applied in place (scene tensors,
    momentum and moments are updated; gradients are written to `grads` only
    when given).
    sghmc: lr, friction (0.1), k (100), t (0.995), burn_in, noise, seed, step.
    adam: beta1, beta2, eps, t and per array of STEP_ARRAYS: m[name], v[name]
    (moment tensors), lr[name], lo[name], hi[name] (defaults +-3e38)."""
    cams = camera_batch(cams)
    n = scene["means"].shape[0]
    E = n * len(cams)
    if deterministic:
        mode |= BWD_DETERMINISTIC
        need = int(lib().sss_render_bwd_workspace_det(E, bins.n_pairs, cams.n_tiles))
    else:
        need = int(lib().sss_render_bwd_workspace(E, cams.n_tiles))
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need // 4, dtype=torch.float32, device=scene["means"].device)
    st = Step()
    for k, name in enumerate(("means", "scales", "quats", "nu", "opacity", "sh")):
        st.params[k] = scene[name].data_ptr()
    _need(momentum, torch.float32, "momentum")
    st.momentum = momentum.data_ptr()
    st.sghmc = SghmcOpts(sghmc["lr"], sghmc.get("friction", 0.1), sghmc.get("k", 100.0), sghmc.get("t", 0.995),
                         int(sghmc.get("burn_in", False)), int(sghmc.get("noise", True)), sghmc.get("seed", 0),
                         sghmc.get("step", 0))
    if adam is not None:
        st.adam = 1
        st.beta1, st.beta2, st.eps = adam.get("beta1", 0.9), adam.get("beta2", 0.999), adam.get("eps", 1e-15)
        st.t = int(adam["t"])
        for k, name in enumerate(STEP_ARRAYS):
            _need(adam["m"][name], torch.float32, f"m[{name}]")
            _need(adam["v"][name], torch.float32, f"v[{name}]")
            st.m[k] = adam["m"][name].data_ptr()
            st.v[k] = adam["v"][name].data_ptr()
            st.lr[k] = adam["lr"][name]
            st.lo[k] = adam.get("lo", {}).get(name, -3.0e38)
            st.hi[k] = adam.get("hi", {}).get(name, 3.0e38)
    s = scene_struct(scene)
    p = proj.struct()
    b = bins.struct()
    g = None
    if grads is not None:
        g = Grads(*(grads[k].data_ptr() for k in ("means", "scales", "quats", "nu", "opacity", "sh")), 1, 0)
    _check(lib().sss_render_bwd_step(ctypes.byref(s), ctypes.byref(p), ctypes.byref(b), cams.array, len(cams),
                                     ctypes.byref(render_opts(opts)), mode, loss, _ptr(dl_or_target), _ptr(image),
                                     _ptr(n_contrib), _ptr(image_out), _ptr(loss_out),
                                     ctypes.byref(g) if g is not None else None, ctypes.byref(st), _ptr(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)), "sss_render_bwd_step")
    return ws


# ---------------------------------------------------------------------------
# kernel timing
# ---------------------------------------------------------------------------
def timing_enable(on: bool = True):
    _check(lib().sss_timing_enable(int(on)), "sss_timing_enable")


def timing_reset():
    lib().sss_timing_reset()


def timing_read() -> dict:
    """{kernel name: (launches, total ms)} since the last reset (waits for the events)."""
    buf = (KernelTime * 64)()
    k = lib().sss_timing_read(buf, 64)
    if k < 0:
        _check(k, "sss_timing_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(k)}


# ---------------------------------------------------------------------------
# streaming copy (a measurement aid)
# ---------------------------------------------------------------------------
def stream_copy(src, dst, stream=None):
    """dst <- src with the library's streaming access pattern (same-size
    contiguous CUDA tensors, 16-byte aligned, a multiple of 16 bytes)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous CUDA tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    _check(lib().sss_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "sss_stream_copy")


# ---------------------------------------------------------------------------
# recycling
# ---------------------------------------------------------------------------
def relocate(scene, states=(), dead_opacity=0.005, max_fraction=0.05, seed=0, step=0, ws=None, stream=None,
             want_count=True):
    """In-place recycling step on the scene tensors; `states` are [n, w]
    tensors (momentum, Adam moments) whose moved rows are zeroed.  Returns
    the number of components moved (waits for the stream) or None."""
    n = scene["means"].shape[0]
    s = scene_struct(scene)
    st = (StateArray * max(1, len(states)))()
    for k, a in enumerate(states):
        _need(a, torch.float32, "state")
        st[k] = StateArray(a.data_ptr(), a.numel() // n, 0)
    need = int(lib().sss_relocate_workspace(n, max_fraction))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=scene["means"].device)
    o = RelocateOpts(dead_opacity, max_fraction, seed, step)
    moved = ctypes.c_int64(0)
    _check(lib().sss_relocate(ctypes.byref(s), st, len(states), ctypes.byref(o), _ptr(ws), ws.numel(),
                              ctypes.byref(moved) if want_count else None, _stream(stream)), "sss_relocate")
    return int(moved.value) if want_count else None


# ---------------------------------------------------------------------------
# loss
# ---------------------------------------------------------------------------
def loss(image, target, cams, lambda_dssim=0.2, dl_dimage=None, loss_out=None, ws=None, stream=None):
    """(1 - lambda) L1 + lambda (1 - SSIM) over all views; returns dL/dimage
    (and adds L into loss_out when given)."""
    cams = camera_batch(cams)
    P = cams.n_pixels
    _need(image, torch.float32, "image")
    _need(target, torch.float32, "target")
    dl_dimage = torch.empty_like(image) if dl_dimage is None else dl_dimage
    need = int(lib().sss_loss_workspace(P))
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(max(need // 4, 1), dtype=torch.float32, device=image.device)
    _check(lib().sss_loss(_ptr(image), _ptr(target), cams.array, len(cams), lambda_dssim, _ptr(dl_dimage),
                          _ptr(loss_out), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)), "sss_loss")
    return dl_dimage


def regularise(opacity, scales, eps_opacity, eps_sigma, d_opacity=None, d_scales=None, loss_out=None, stream=None):
    """eps_o sum |o| + eps_sigma sum sqrt(eig Sigma) (= sum |s|): adds the
    gradients into d_opacity / d_scales and the value into loss_out (each
    optional, device tensors)."""
    _need(opacity, torch.float32, "opacity")
    _need(scales, torch.float32, "scales")
    n = opacity.shape[0]
    _check(lib().sss_regularise(_ptr(opacity), _ptr(scales), n, eps_opacity, eps_sigma, _ptr(d_opacity),
                                _ptr(d_scales), _ptr(loss_out), _stream(stream)), "sss_regularise")
