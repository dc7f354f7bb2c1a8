"""Python binding of libniv (the C interface in include/niv.h).

Marshalling only: device memory comes from torch tensors, streams from
torch's current stream; every step of the method runs in the library's HIP
kernels.  There is no CPU fallback: importing works without a GPU, but any
call that needs the library raises if libniv.so is missing.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libniv.so")

(NIV_OK, NIV_ERR_INVALID_ARG, NIV_ERR_UNSUPPORTED, NIV_ERR_HIP, NIV_ERR_WORKSPACE, NIV_ERR_STATE,
 NIV_ERR_NONFINITE) = range(7)
FP32, FP16, BF16 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "fp16": FP16, "bf16": BF16}
FLAG_OUTSIDE, FLAG_BAD_INPUT, FLAG_BAD_OUTPUT, FLAG_FALLBACK, FLAG_NEG_OUTPUT = 1, 2, 4, 8, 16


class NivError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {status_string(status)} (status {status})")
        self.status = status


class Config(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("log2_T", C.c_int32), ("n_features", C.c_int32),
                ("base_res", C.c_double), ("per_level_scale", C.c_double),
                ("sh_bands", C.c_int32), ("n_extra", C.c_int32), ("extra_bands", C.c_int32),
                ("width", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32),
                ("aabb_min", C.c_double * 3), ("aabb_max", C.c_double * 3),
                ("pos_bands", C.c_int32)]


class Frame(C.Structure):
    _fields_ = [("count", C.c_int64), ("pos", C.c_void_p), ("nrm", C.c_void_p),
                ("albedo", C.c_void_p), ("mask", C.c_void_p),
                ("extra_values", C.c_float * 4), ("model", C.c_void_p),
                ("out_E", C.c_void_p), ("out_L", C.c_void_p), ("out_flags", C.c_void_p),
                ("out_inputs", C.c_void_p), ("in_flags", C.c_void_p), ("scene", C.c_void_p)]


class HalfFrame(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("pos", C.c_void_p),
                ("nrm", C.c_void_p), ("albedo", C.c_void_p), ("mask", C.c_void_p),
                ("extra_values", C.c_float * 4), ("model", C.c_void_p), ("half_E", C.c_void_p),
                ("half_flags", C.c_void_p), ("out_E", C.c_void_p), ("out_L", C.c_void_p),
                ("out_flags", C.c_void_p)]


class UpsampleParams(C.Structure):
    _fields_ = [("sigma_px", C.c_float), ("sigma_pos", C.c_float), ("normal_power", C.c_int32)]


class AoParams(C.Structure):
    _fields_ = [("rays", C.c_int32), ("radius", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


class Fallback(C.Structure):
    _fields_ = [("flag_mask", C.c_uint32), ("spp", C.c_int32), ("bounces", C.c_int32),
                ("mc_flags", C.c_int32), ("seed", C.c_uint64)]


class TuneResult(C.Structure):
    _fields_ = [("n", C.c_int32), ("block", C.c_int32 * 24), ("blocks_per_cu", C.c_int32 * 24),
                ("xcd_order", C.c_int32 * 24), ("ms", C.c_float * 24), ("chosen_block", C.c_int32),
                ("chosen_blocks_per_cu", C.c_int32), ("chosen_xcd_order", C.c_int32),
                ("chosen_ms", C.c_float)]


class Batch(C.Structure):
    _fields_ = [("count", C.c_int64), ("x", C.c_void_p), ("nrm", C.c_void_p),
                ("extra", C.c_void_p), ("target", C.c_void_p), ("valid", C.c_void_p)]


class TrainState(C.Structure):
    _fields_ = [("params", C.c_void_p), ("grads", C.c_void_p), ("adam_m", C.c_void_p),
                ("adam_v", C.c_void_p), ("model", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_int64), ("loss", C.c_void_p)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("step", C.c_int64)]


_lib = None
NOALLOC_MAX_FLAGGED = 1 << 20   # NIV_NOALLOC_MAX_FLAGGED
MC_NEE, MC_EMIT_ON_HIT, MC_INCLUDE_DIRECT, MC_DIRECT_AT_ORIGIN = 1, 2, 4, 8


def lib():
    """The loaded libniv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.niv_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.niv_destroy.argtypes = [vp]
        L.niv_destroy.restype = None
        L.niv_sizes.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64)]
        L.niv_level_info.argtypes = [vp, vp, vp, vp, vp]
        L.niv_prepare.argtypes = [vp, vp, vp, C.c_int, vp]
        L.niv_query.argtypes = [vp, C.POINTER(Frame), C.c_int32, C.c_int, vp]
        L.niv_status_string.argtypes = [C.c_int]
        L.niv_status_string.restype = C.c_char_p
        L.niv_upsample.argtypes = [vp, C.POINTER(HalfFrame), C.POINTER(UpsampleParams), vp]
        L.niv_query_half.argtypes = [vp, C.POINTER(HalfFrame), C.POINTER(UpsampleParams), C.c_int, vp]
        L.niv_fallback_sizes.argtypes = [vp, C.c_int64, C.POINTER(C.c_int64)]
        L.niv_probe_gather.argtypes = [C.c_int32, C.c_int32, vp, vp, vp]
        L.niv_probe_encode.argtypes = [vp, C.POINTER(Frame), C.c_int, vp]
        L.niv_corner_indices.argtypes = [vp, C.c_int, C.c_int32, vp, vp, C.c_int64, vp, vp]
        L.niv_query_fallback.argtypes = [vp, C.POINTER(Frame), C.c_int32, C.c_int,
                                         C.POINTER(Fallback), vp, C.c_int64, vp]
        L.niv_query_fallback_noalloc.argtypes = [vp, C.POINTER(Frame), C.c_int32, C.c_int,
                                                 C.POINTER(Fallback), C.c_int64, vp]
        L.niv_autotune.argtypes = [vp, C.POINTER(Frame), C.c_int32, C.c_int, vp,
                                   C.POINTER(TuneResult)]
        L.niv_set_tune.argtypes = [vp, C.c_int, C.c_int32, C.c_int32, C.c_int32]
        L.niv_graph_capture.argtypes = [vp, C.POINTER(Frame), C.c_int32, C.c_int,
                                        C.POINTER(Fallback), vp, C.c_int64, C.POINTER(vp)]
        L.niv_graph_launch.argtypes = [vp, vp]
        L.niv_graph_destroy.argtypes = [vp]
        L.niv_graph_destroy.restype = None
        L.niv_train_sizes.argtypes = [vp, C.c_int, C.c_int64, C.POINTER(C.c_int64)]
        L.niv_backward.argtypes = [vp, C.POINTER(Batch), C.POINTER(TrainState), C.c_int, vp]
        L.niv_adam_update.argtypes = [vp, C.POINTER(TrainState), C.POINTER(Adam), vp]
        L.niv_train_step.argtypes = [vp, C.POINTER(Batch), C.POINTER(TrainState), C.POINTER(Adam),
                                     C.c_int, vp]
        L.niv_train_status.argtypes = [C.POINTER(TrainState), vp]
        L.niv_lr_schedule.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                      C.POINTER(C.c_double)]
        L.niv_init_params.argtypes = [vp, vp, C.c_uint64, C.c_float, C.c_float, vp]
        L.mc_scene_create.argtypes = [vp, C.c_int32, C.POINTER(vp)]
        L.mc_scene_destroy.argtypes = [vp]
        L.mc_scene_destroy.restype = None
        L.mc_irradiance.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_uint64, vp, vp, vp, vp, vp, vp]
        L.mc_scene_set_motion.argtypes = [vp, vp]
        L.mc_sample_points_t.argtypes = [vp, vp, vp, C.c_int64, C.c_int64, C.c_uint64, vp, vp, vp, vp]
        L.mc_irradiance_at.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_uint64, vp, vp, vp, vp, vp, vp]
        L.mc_sample_points.argtypes = [vp, vp, vp, C.c_int64, C.c_int64, C.c_uint64, vp, vp, vp]
        L.niv_ao_create.argtypes = [vp, C.c_int64, C.POINTER(vp)]
        L.niv_ao_destroy.argtypes = [vp]
        L.niv_ao_destroy.restype = None
        L.niv_ao_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.niv_ao_apply.argtypes = [vp, C.POINTER(AoParams), C.c_int64, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def status_string(s):
    return lib().niv_status_string(int(s)).decode()


def _check(status, what):
    if status != NIV_OK:
        raise NivError(status, what)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def probe_gather(mode, n, table, out):
    """niv_probe_gather: one pass of n x 128 gathers in pattern `mode`
    (measurement); table: 8 MiB device tensor, out: 2048 x 256 words."""
    _check(lib().niv_probe_gather(int(mode), int(n), _ptr(table), _ptr(out), _stream()),
           "niv_probe_gather")


def lr_schedule(step, hold_steps, total_steps, lr0=1e-2, lr1=1e-4):
    """niv_lr_schedule: the Sec. 4.5 learning rate of a 1-based step."""
    out = C.c_double()
    _check(lib().niv_lr_schedule(int(step), int(hold_steps), int(total_steps), float(lr0),
                                 float(lr1), C.byref(out)), "niv_lr_schedule")
    return out.value


def make_config(d) -> Config:
    c = Config()
    for k in ("n_levels", "log2_T", "n_features", "sh_bands", "n_extra", "extra_bands",
              "width", "n_hidden", "n_out"):
        setattr(c, k, int(d[k]))
    c.pos_bands = int(d.get("pos_bands", 0))
    c.base_res = float(d["base_res"])
    c.per_level_scale = float(d["per_level_scale"])
    c.aabb_min = (C.c_double * 3)(*[float(x) for x in d["aabb_min"]])
    c.aabb_max = (C.c_double * 3)(*[float(x) for x in d["aabb_max"]])
    return c


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


class NIV:
    """A model shape (niv_create); parameters live in caller-owned tensors."""

    def __init__(self, cfg):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        h = C.c_void_p()
        _check(lib().niv_create(C.byref(self._c), C.byref(h)), "niv_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.niv_destroy(h)
            self._h = None

    # ---------------------------------------------------------- sizes
    def sizes(self, prec="fp16"):
        n_p, n_g, nb = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().niv_sizes(self._h, _prec(prec), C.byref(n_p), C.byref(n_g), C.byref(nb)),
               "niv_sizes")
        return n_p.value, n_g.value, nb.value

    @property
    def n_params(self):
        n_p, n_g = C.c_int64(), C.c_int64()
        _check(lib().niv_sizes(self._h, FP32, C.byref(n_p), C.byref(n_g), None), "niv_sizes")
        return n_p.value

    @property
    def n_grid_values(self):
        n_p, n_g = C.c_int64(), C.c_int64()
        _check(lib().niv_sizes(self._h, FP32, C.byref(n_p), C.byref(n_g), None), "niv_sizes")
        return n_g.value

    def mat_shapes(self):
        """(out, in) of every weight matrix, input layer first (row-major
        blocks after the grid in the parameter vector)."""
        c = self.cfg
        W = c["width"]
        return [(W, self.input_dim)] + [(W, W)] * (c["n_hidden"] - 1) + [(c["n_out"], W)]

    def init_params(self, seed, grid_lo=-1e-4, grid_hi=1e-4, out=None, device="cuda"):
        """niv_init_params: seeded FP32 master parameters on the device (grid
        uniform on [grid_lo, grid_hi), weights Xavier-uniform)."""
        if out is None:
            out = torch.empty(self.n_params, dtype=torch.float32, device=device)
        assert out.is_cuda and out.dtype == torch.float32 and out.numel() == self.n_params
        _check(lib().niv_init_params(self._h, _ptr(out), C.c_uint64(int(seed)), float(grid_lo),
                                     float(grid_hi), _stream()), "niv_init_params")
        return out

    def level_info(self):
        import numpy as np
        L = self.cfg["n_levels"]
        res = np.zeros(L, np.int64)
        dense = np.zeros(L, np.int32)
        off = np.zeros(L, np.int64)
        size = np.zeros(L, np.int64)
        _check(lib().niv_level_info(self._h, res.ctypes.data, dense.ctypes.data, off.ctypes.data,
                                    size.ctypes.data), "niv_level_info")
        return dict(res=res, dense=dense.astype(bool), offset=off, size=size)

    # ---------------------------------------------------------- model
    def prepare(self, params, prec="fp16", out=None):
        """Prepared model for queries at `prec` from FP32 master parameters."""
        assert params.is_cuda and params.dtype == torch.float32 and params.is_contiguous()
        assert params.numel() == self.n_params
        nb = self.sizes(prec)[2]
        if out is None:
            out = torch.empty(nb, dtype=torch.uint8, device=params.device)
        assert out.numel() >= nb and out.data_ptr() % 256 == 0
        _check(lib().niv_prepare(self._h, _ptr(params), _ptr(out), _prec(prec), _stream()),
               "niv_prepare")
        return out

    def frame(self, pos, nrm, model, albedo=None, mask=None, extra=(), out_E=None, out_L=None,
              out_flags=None, want_L=True, want_flags=True, out_inputs=None, in_flags=None,
              scene=None):
        """Builds a niv_frame (and the output tensors) for one G-buffer."""
        n = pos.numel() // 3
        dev = pos.device
        for t in (pos, nrm, albedo):
            if t is not None:
                assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.is_contiguous()
        if out_E is None:
            out_E = torch.empty(pos.shape, dtype=torch.float32, device=dev)
        if out_L is None and want_L and albedo is not None:
            out_L = torch.empty(pos.shape, dtype=torch.float32, device=dev)
        if out_flags is None and want_flags:
            out_flags = torch.empty(pos.shape[:-1], dtype=torch.uint8, device=dev)
        f = Frame()
        f.count = n
        f.pos, f.nrm, f.albedo, f.mask = (_ptr(pos).value, _ptr(nrm).value,
                                          _ptr(albedo).value, _ptr(mask).value)
        ev = list(extra) + [0.0] * (4 - len(extra))
        f.extra_values = (C.c_float * 4)(*[float(x) for x in ev])
        f.model = _ptr(model).value
        f.out_E = _ptr(out_E).value
        f.out_L = _ptr(out_L).value
        f.out_flags = _ptr(out_flags).value
        f.out_inputs = _ptr(out_inputs).value
        f.in_flags = _ptr(in_flags).value
        f.scene = scene._h.value if scene is not None else None
        return f, (out_E, out_L, out_flags)

    def query_frames(self, frames, prec="fp16"):
        arr = (Frame * len(frames))(*frames)
        _check(lib().niv_query(self._h, arr, len(frames), _prec(prec), _stream()), "niv_query")

    # ---------------------------------------------------------- half resolution
    def half_frame(self, width, height, pos, nrm, model=None, albedo=None, mask=None, extra=(),
                   half_E=None, want_L=True, want_flags=True):
        """A niv_half_frame (and its tensors) for one full-resolution G-buffer
        of height x width pixels: half_E / half_flags at the samples (2x, 2y),
        out_E / out_L / out_flags at every pixel."""
        dev = pos.device
        hw, hh = (width + 1) // 2, (height + 1) // 2
        assert pos.numel() == nrm.numel() == 3 * width * height
        if half_E is None:
            half_E = torch.empty((hh * hw, 3), dtype=torch.float32, device=dev)
        half_flags = torch.empty(hh * hw, dtype=torch.uint8, device=dev) if want_flags else None
        out_E = torch.empty((width * height, 3), dtype=torch.float32, device=dev)
        out_L = (torch.empty((width * height, 3), dtype=torch.float32, device=dev)
                 if (want_L and albedo is not None) else None)
        out_flags = torch.empty(width * height, dtype=torch.uint8, device=dev) if want_flags else None
        f = HalfFrame()
        f.width, f.height = int(width), int(height)
        f.pos, f.nrm, f.albedo, f.mask = (_ptr(pos).value, _ptr(nrm).value, _ptr(albedo).value,
                                          _ptr(mask).value)
        ev = list(extra) + [0.0] * (4 - len(extra))
        f.extra_values = (C.c_float * 4)(*[float(x) for x in ev])
        f.model = _ptr(model).value
        f.half_E, f.half_flags = _ptr(half_E).value, _ptr(half_flags).value
        f.out_E, f.out_L, f.out_flags = _ptr(out_E).value, _ptr(out_L).value, _ptr(out_flags).value
        return f, dict(half_E=half_E, half_flags=half_flags, E=out_E, L=out_L, flags=out_flags)

    @staticmethod
    def upsample_params(sigma_px=1.0, sigma_pos=0.1, normal_power=8):
        return UpsampleParams(float(sigma_px), float(sigma_pos), int(normal_power))

    def upsample(self, f, params=None):
        """niv_upsample: joint bilateral upsampling of f.half_E (Sec. 4.4)."""
        p = params or self.upsample_params()
        _check(lib().niv_upsample(self._h, C.byref(f), C.byref(p), _stream()), "niv_upsample")

    def query_half(self, f, prec="fp16", params=None):
        """niv_query_half: the query at a quarter of the pixels, then upsampling."""
        p = params or self.upsample_params()
        _check(lib().niv_query_half(self._h, C.byref(f), C.byref(p), _prec(prec), _stream()),
               "niv_query_half")

    def corner_indices(self, pos, model, prec="fp32", training=False):
        """niv_corner_indices: grid entries [n, L, 8] (int32 tensor) read by the
        query's encoding at `prec` for each position."""
        n = pos.numel() // 3
        out = torch.empty((n, self.cfg["n_levels"], 8), dtype=torch.int32, device=pos.device)
        _check(lib().niv_corner_indices(self._h, _prec(prec), int(bool(training)), _ptr(model), _ptr(pos),
                                        n, _ptr(out), _stream()), "niv_corner_indices")
        return out

    def probe_encode(self, frame, prec="fp16"):
        """niv_probe_encode: the query's encoding stage alone on one frame
        (measurement; writes one word per pixel into the frame's out_E)."""
        _check(lib().niv_probe_encode(self._h, C.byref(frame), _prec(prec), _stream()),
               "niv_probe_encode")

    def fallback_workspace(self, max_flagged, device="cuda"):
        nb = C.c_int64()
        _check(lib().niv_fallback_sizes(self._h, int(max_flagged), C.byref(nb)), "niv_fallback_sizes")
        return torch.empty(nb.value, dtype=torch.uint8, device=device)

    @staticmethod
    def fallback(flag_mask=FLAG_OUTSIDE | FLAG_BAD_OUTPUT, spp=64, bounces=3, mc_flags=MC_NEE,
                 seed=0):
        return Fallback(int(flag_mask), int(spp), int(bounces), int(mc_flags), int(seed))

    def query_fallback(self, frames, prec, fb, workspace):
        """niv_query_fallback: query, then Monte Carlo for flagged pixels."""
        arr = (Frame * len(frames))(*frames)
        _check(lib().niv_query_fallback(self._h, arr, len(frames), _prec(prec), C.byref(fb),
                                        _ptr(workspace), workspace.numel(), _stream()),
               "niv_query_fallback")

    def query_fallback_noalloc(self, frames, prec, fb, max_flagged):
        """niv_query_fallback_noalloc: as query_fallback, with the list in the
        library's fixed scratch (at most NOALLOC_MAX_FLAGGED entries)."""
        arr = (Frame * len(frames))(*frames)
        _check(lib().niv_query_fallback_noalloc(self._h, arr, len(frames), _prec(prec), C.byref(fb),
                                                int(max_flagged), _stream()),
               "niv_query_fallback_noalloc")

    def autotune(self, frames, prec):
        """Times the launch shapes on these frames, keeps the fastest."""
        arr = (Frame * len(frames))(*frames)
        r = TuneResult()
        _check(lib().niv_autotune(self._h, arr, len(frames), _prec(prec), _stream(), C.byref(r)),
               "niv_autotune")
        return {"candidates": [(r.block[k], r.blocks_per_cu[k], r.xcd_order[k], r.ms[k])
                               for k in range(r.n)],
                "block": r.chosen_block, "blocks_per_cu": r.chosen_blocks_per_cu,
                "xcd_order": r.chosen_xcd_order, "ms": r.chosen_ms}

    def set_tune(self, prec, block, blocks_per_cu, xcd_order):
        """Pins the launch shape of later queries at `prec` (niv_set_tune)."""
        _check(lib().niv_set_tune(self._h, _prec(prec), int(block), int(blocks_per_cu),
                                  int(xcd_order)), "niv_set_tune")

    def capture(self, frames, prec, fb=None, workspace=None):
        """A HIP graph of one frame's query (and fallback); see Graph."""
        return Graph(self, frames, prec, fb, workspace)

    @property
    def input_dim(self):
        c = self.cfg
        pb = c.get("pos_bands", 0)
        return (c["n_levels"] * c["n_features"] + (3 + 6 * pb if pb > 0 else 0) + c["sh_bands"] ** 2
                + c["n_extra"] * 2 * c["extra_bands"])

    def query(self, pos, nrm, model, prec="fp16", albedo=None, mask=None, extra=(),
              want_flags=True, want_inputs=False):
        """E, L (= albedo * E / pi or None) and flags (and the encoded inputs if
        asked) for one G-buffer."""
        inputs = None
        if want_inputs:
            inputs = torch.empty((pos.numel() // 3, self.input_dim), dtype=torch.float32,
                                 device=pos.device)
        f, outs = self.frame(pos, nrm, model, albedo=albedo, mask=mask, extra=extra,
                             want_flags=want_flags, out_inputs=inputs)
        self.query_frames([f], prec)
        return outs + (inputs,) if want_inputs else outs


class DynamicAO:
    """Dynamic ambient occlusion (Sec. 4.4): a hierarchy over the dynamic
    triangles `tris` [m,3,3] (host array; niv_ao_create) and its pass over a
    frame's pixels (niv_ao_apply)."""

    def __init__(self, tris):
        import numpy as np
        t = np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 9)
        h = C.c_void_p()
        _check(lib().niv_ao_create(t.ctypes.data if t.size else None, t.shape[0], C.byref(h)),
               "niv_ao_create")
        self._h = h
        self.n_tris = t.shape[0]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.niv_ao_destroy(h)
            self._h = None

    def info(self):
        """(nodes, depth) of the hierarchy."""
        n, d = C.c_int32(), C.c_int32()
        _check(lib().niv_ao_info(self._h, C.byref(n), C.byref(d)), "niv_ao_info")
        return n.value, d.value

    def apply(self, pos, nrm, rays, radius, eps, seed, mask=None, E=None, L=None, vis=None):
        """Visibility V of each pixel (returned, [n] float) and, in place, E and
        L times V."""
        n = pos.numel() // 3
        if vis is None:
            vis = torch.empty(n, dtype=torch.float32, device=pos.device)
        p = AoParams(int(rays), float(radius), float(eps), int(seed))
        _check(lib().niv_ao_apply(self._h, C.byref(p), n, _ptr(pos), _ptr(nrm), _ptr(mask), _ptr(E),
                                  _ptr(L), _ptr(vis), _stream()), "niv_ao_apply")
        return vis


class McScene:
    """A scene on the device (mc_scene_create) for the Monte Carlo estimator
    of Eq. 1 and the training-point sampler.  `prims` is a numpy structured
    array of 64-byte primitive records (see niv_synth.scene)."""

    def __init__(self, prims):
        import numpy as np
        self.prims = np.ascontiguousarray(prims)
        assert self.prims.dtype.itemsize == 64
        h = C.c_void_p()
        _check(lib().mc_scene_create(self.prims.ctypes.data, len(self.prims), C.byref(h)),
               "mc_scene_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.mc_scene_destroy(h)
            self._h = None

    def set_motion(self, motion):
        """mc_scene_set_motion: primitive k translated by t * motion[k] (Sec. 6);
        None makes the scene static again."""
        import numpy as np
        if motion is None:
            _check(lib().mc_scene_set_motion(self._h, None), "mc_scene_set_motion")
            self.motion = None
            return
        m = np.ascontiguousarray(motion, dtype=np.float32).reshape(len(self.prims), 3)
        _check(lib().mc_scene_set_motion(self._h, m.ctypes.data), "mc_scene_set_motion")
        self.motion = m

    def irradiance(self, x, nrm, spp, bounces, flags, seed, out=None, t=None):
        """(E [n,3] f64, var [n,3] f64, back faces [n] i32, valid [n] u8);
        t: scene variable per point (device float [n]) or None."""
        n = x.numel() // 3
        dev = x.device
        if out is None:
            out = (torch.empty((n, 3), dtype=torch.float64, device=dev),
                   torch.empty((n, 3), dtype=torch.float64, device=dev),
                   torch.empty(n, dtype=torch.int32, device=dev),
                   torch.empty(n, dtype=torch.uint8, device=dev))
        E, var, bf, vd = out
        _check(lib().mc_irradiance_at(self._h, _ptr(x), _ptr(nrm), _ptr(t), n, int(spp), int(bounces),
                                      int(flags), C.c_uint64(int(seed)), _ptr(E), None, _ptr(var),
                                      _ptr(bf), _ptr(vd), _stream()), "mc_irradiance_at")
        return out

    def targets(self, x, nrm, spp, bounces, seed, flags=1, out=None, t=None):
        """Training targets: (E [n,3] float32, valid [n] uint8)."""
        n = x.numel() // 3
        if out is None:
            out = (torch.empty((n, 3), dtype=torch.float32, device=x.device),
                   torch.empty(n, dtype=torch.uint8, device=x.device))
        E32, vd = out
        _check(lib().mc_irradiance_at(self._h, _ptr(x), _ptr(nrm), _ptr(t), n, int(spp), int(bounces),
                                      int(flags), C.c_uint64(int(seed)), None, _ptr(E32), None,
                                      None, _ptr(vd), _stream()), "mc_irradiance_at")
        return out

    def sample_points(self, lo, hi, count, n_surface, seed, device="cuda", out=None, with_t=False):
        """Training points: (x [count,3], n [count,3]) float32 on the device,
        and with with_t a scene variable per point (t [count], uniform)."""
        lo_a = (C.c_double * 3)(*[float(v) for v in lo])
        hi_a = (C.c_double * 3)(*[float(v) for v in hi])
        if out is None:
            out = (torch.empty((count, 3), dtype=torch.float32, device=device),
                   torch.empty((count, 3), dtype=torch.float32, device=device))
            if with_t:
                out = out + (torch.empty(count, dtype=torch.float32, device=device),)
        x, n = out[0], out[1]
        t = out[2] if with_t else None
        _check(lib().mc_sample_points_t(self._h, lo_a, hi_a, int(count), int(n_surface),
                                        C.c_uint64(int(seed)), _ptr(x), _ptr(n), _ptr(t), _stream()),
               "mc_sample_points_t")
        return (x, n, t) if with_t else (x, n)


class Graph:
    """niv_graph_capture / niv_graph_launch: the frame's launches replayed
    with the same buffers (whose contents may change)."""

    def __init__(self, niv, frames, prec, fb, workspace):
        self._keep = (niv, frames, workspace)
        arr = (Frame * len(frames))(*frames)
        g = C.c_void_p()
        _check(lib().niv_graph_capture(niv._h, arr, len(frames), _prec(prec),
                                       C.byref(fb) if fb is not None else None,
                                       _ptr(workspace), workspace.numel() if workspace is not None else 0,
                                       C.byref(g)), "niv_graph_capture")
        self._g = g

    def launch(self):
        _check(lib().niv_graph_launch(self._g, _stream()), "niv_graph_launch")

    def __del__(self):
        g = getattr(self, "_g", None)
        if g is not None and g.value and _lib is not None:
            _lib.niv_graph_destroy(g)
            self._g = None


class Trainer:
    """Training state for one model (niv_backward / niv_adam_update /
    niv_train_step): FP32 master parameters, gradient, Adam moments, the
    prepared model of the training precision and the scratch buffer, all
    torch tensors on the device."""

    def __init__(self, niv, params, prec="fp16", max_batch=1 << 18):
        assert params.is_cuda and params.dtype == torch.float32 and params.is_contiguous()
        self.niv, self.prec = niv, _prec(prec)
        dev = params.device
        self.params = params
        self.grads = torch.zeros_like(params)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.model = niv.prepare(params, self.prec)
        nb = C.c_int64()
        _check(lib().niv_train_sizes(niv._h, self.prec, int(max_batch), C.byref(nb)), "niv_train_sizes")
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.max_batch = max_batch
        self.step_count = 0
        st = TrainState()
        st.params, st.grads = params.data_ptr(), self.grads.data_ptr()
        st.adam_m, st.adam_v = self.m.data_ptr(), self.v.data_ptr()
        st.model, st.workspace = self.model.data_ptr(), self.workspace.data_ptr()
        st.workspace_bytes = nb.value
        st.loss = self.loss.data_ptr()
        self._st = st

    def _batch(self, x, nrm, target, valid=None, extra=None):
        n = x.numel() // 3
        assert n <= self.max_batch
        b = Batch()
        b.count = n
        b.x, b.nrm, b.target = x.data_ptr(), nrm.data_ptr(), target.data_ptr()
        b.extra = extra.data_ptr() if extra is not None else None
        b.valid = valid.data_ptr() if valid is not None else None
        return b

    def backward(self, x, nrm, target, valid=None, extra=None):
        """Loss (device scalar) and gradient (self.grads) of one batch."""
        b = self._batch(x, nrm, target, valid, extra)
        _check(lib().niv_backward(self.niv._h, C.byref(b), C.byref(self._st), self.prec, _stream()),
               "niv_backward")
        return self.loss

    def status(self):
        """niv_train_status: waits for the stream; False if the last step's loss
        or gradient was not finite (its update was skipped), else True."""
        st = lib().niv_train_status(C.byref(self._st), _stream())
        if st == NIV_ERR_NONFINITE:
            return False
        _check(st, "niv_train_status")
        return True

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, step=None):
        self.step_count = step if step is not None else self.step_count + 1
        ad = Adam(lr, beta1, beta2, eps, self.step_count)
        _check(lib().niv_adam_update(self.niv._h, C.byref(self._st), C.byref(ad), _stream()),
               "niv_adam_update")

    def step(self, x, nrm, target, lr, valid=None, extra=None, beta1=0.9, beta2=0.999, eps=1e-8):
        """One training step; returns the batch loss (device scalar)."""
        b = self._batch(x, nrm, target, valid, extra)
        self.step_count += 1
        ad = Adam(lr, beta1, beta2, eps, self.step_count)
        _check(lib().niv_train_step(self.niv._h, C.byref(b), C.byref(self._st), C.byref(ad),
                                    self.prec, _stream()), "niv_train_step")
        return self.loss
