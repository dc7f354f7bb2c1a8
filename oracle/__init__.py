"""FP64 CPU oracle for the Neural Irradiance Volume hot path.

TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference that the GPU
library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the GPU library; both read the same input data.

The arithmetic lives in niv_oracle.c (plain C, double precision, OpenMP);
this module is marshalling only.  Each wrapper names the passage of the paper
it follows.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "niv_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MC_NEE, MC_EMIT_ON_HIT, MC_INCLUDE_DIRECT, MC_DIRECT_AT_ORIGIN = 1, 2, 4, 8
FLAG_OUTSIDE, FLAG_BAD_INPUT, FLAG_BAD_OUTPUT, FLAG_NEG_OUTPUT = 1, 2, 4, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Config(C.Structure):
    _fields_ = [("n_levels", C.c_int), ("log2_T", C.c_int), ("n_features", C.c_int),
                ("base_res", C.c_double), ("per_level_scale", C.c_double),
                ("sh_bands", C.c_int), ("n_extra", C.c_int), ("extra_bands", C.c_int),
                ("width", C.c_int), ("n_hidden", C.c_int), ("n_out", C.c_int),
                ("aabb_min", C.c_double * 3), ("aabb_max", C.c_double * 3),
                ("pos_bands", C.c_int)]


def make_config(**kw) -> Config:
    c = Config()
    for k, v in kw.items():
        if k in ("aabb_min", "aabb_max"):
            setattr(c, k, (C.c_double * 3)(*[float(x) for x in v]))
        else:
            setattr(c, k, v)
    return c


def _P(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_LIB_PATH)
        cp = C.POINTER(Config)
        i64p, dp, fp, u8p = (C.POINTER(C.c_int64), C.POINTER(C.c_double),
                             C.POINTER(C.c_float), C.POINTER(C.c_uint8))
        L.orc_level_table.argtypes = [cp, i64p, C.POINTER(C.c_int), i64p, i64p]
        L.orc_level_table.restype = C.c_int64
        L.orc_input_dim.argtypes = [cp]
        L.orc_input_dim.restype = C.c_int
        L.orc_n_params.argtypes = [cp]
        L.orc_n_params.restype = C.c_int64
        L.orc_n_grid_values.argtypes = [cp]
        L.orc_n_grid_values.restype = C.c_int64
        L.orc_hash.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_int]
        L.orc_hash.restype = C.c_uint32
        L.orc_dense_index.argtypes = [C.c_int64] * 4
        L.orc_dense_index.restype = C.c_int64
        L.orc_legendre.argtypes = [C.c_int, C.c_int, C.c_double]
        L.orc_legendre.restype = C.c_double
        L.orc_sh.argtypes = [C.c_int, dp, dp]
        L.orc_freq.argtypes = [C.c_int, C.c_double, dp]
        L.orc_query.argtypes = [cp, dp, C.c_int64, fp, fp, fp, fp, u8p, dp, dp, u8p, dp]
        L.orc_corners.argtypes = [cp, fp, i64p, dp]
        L.orc_corners_n.argtypes = [cp, fp, C.c_int64, i64p]
        L.orc_loss_grad.argtypes = [cp, dp, C.c_int64, fp, fp, fp, fp, u8p, C.c_double, dp]
        L.orc_loss_grad.restype = C.c_double
        L.orc_loss.argtypes = [cp, dp, C.c_int64, fp, fp, fp, fp, u8p, C.c_double]
        L.orc_loss.restype = C.c_double
        L.orc_adam.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_int64]
        L.orc_lr.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double]
        L.orc_lr.restype = C.c_double
        L.orc_philox4x64.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                     C.POINTER(C.c_uint64)]
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int]
        L.orc_uniform.restype = C.c_double
        L.orc_init_params.argtypes = [cp, C.c_uint64, C.c_double, C.c_double, fp]
        L.orc_init_params.restype = None
        L.orc_mc_irradiance.argtypes = [C.c_void_p, C.c_int, fp, fp, C.c_void_p, C.c_int64, C.c_int,
                                        C.c_int, C.c_int, C.c_uint64, dp, dp,
                                        C.POINTER(C.c_int32), u8p, fp, fp]
        L.orc_upsample.argtypes = [cp, C.c_int, C.c_int, fp, fp, u8p, fp, dp, C.c_double,
                                   C.c_double, C.c_int, dp, dp, u8p]
        L.orc_upsample.restype = None
        L.orc_sample_points.argtypes = [C.c_void_p, C.c_int, dp, dp, C.c_int64,
                                        C.c_int64, C.c_uint64, fp, fp, fp]
        L.orc_dynamic_ao.argtypes = [fp, C.c_int64, fp, fp, C.c_void_p, C.c_int64, C.c_int,
                                     C.c_double, C.c_double, C.c_uint64, dp]
        L.orc_dynamic_ao.restype = None
        _lib = L
    return _lib


def set_threads(n: int):
    """Limit OpenMP threads (calls omp_set_num_threads through libgomp)."""
    try:
        gomp = C.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(int(n))
    except OSError:
        pass


def _f32(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


# ---------------------------------------------------------------- model
def level_table(cfg: Config):
    """Sec. 4.1: resolutions, dense flags, sizes and offsets per level."""
    L = cfg.n_levels
    res = np.zeros(L, np.int64)
    dense = np.zeros(L, np.int32)
    size = np.zeros(L, np.int64)
    off = np.zeros(L, np.int64)
    total = lib().orc_level_table(C.byref(cfg), _P(res, C.c_int64), _P(dense, C.c_int),
                                  _P(size, C.c_int64), _P(off, C.c_int64))
    return dict(res=res, dense=dense.astype(bool), size=size, offset=off, total=int(total))


def input_dim(cfg: Config) -> int:
    return int(lib().orc_input_dim(C.byref(cfg)))


def n_params(cfg: Config) -> int:
    return int(lib().orc_n_params(C.byref(cfg)))


def n_grid_values(cfg: Config) -> int:
    return int(lib().orc_n_grid_values(C.byref(cfg)))


def mat_shapes(cfg: Config):
    """Weight shapes (out, in): W_0, hidden ..., W_H (Sec. 4.1)."""
    shapes = [(cfg.width, input_dim(cfg))]
    shapes += [(cfg.width, cfg.width)] * (cfg.n_hidden - 1)
    shapes.append((cfg.n_out, cfg.width))
    return shapes


def split_params(cfg: Config, params):
    """Views of the grid block and each weight matrix of a flat vector."""
    g = n_grid_values(cfg)
    out = [params[:g].reshape(-1, cfg.n_features)]
    k = g
    for (o, i) in mat_shapes(cfg):
        out.append(params[k:k + o * i].reshape(o, i))
        k += o * i
    return out


def hash_index(x, y, z, log2_T):
    return int(lib().orc_hash(x, y, z, log2_T))


def dense_index(x, y, z, N):
    return int(lib().orc_dense_index(x, y, z, N))


def legendre(l, m, x):
    return float(lib().orc_legendre(l, m, x))


def sh(bands, n_unit):
    n = np.ascontiguousarray(n_unit, dtype=np.float64)
    out = np.zeros(bands * bands)
    lib().orc_sh(bands, _P(n, C.c_double), _P(out, C.c_double))
    return out


def freq(bands, t):
    out = np.zeros(2 * bands)
    lib().orc_freq(bands, float(t), _P(out, C.c_double))
    return out


def query(cfg: Config, params, pos, nrm, extra=None, albedo=None, mask=None,
          want_x0=False):
    """Sec. 4.4 rendering: E_theta at every point and albedo * E / pi (Eq. 2).
    Returns (E [n, n_out], L [n, n_out], flags [n] uint8[, x0])."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    pos = _f32(pos).reshape(-1, 3)
    nrm = _f32(nrm).reshape(-1, 3)
    n = pos.shape[0]
    ex = None if extra is None else _f32(extra).reshape(n, -1)
    al = None if albedo is None else _f32(albedo).reshape(-1, 3)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    E = np.zeros((n, cfg.n_out))
    Lo = np.zeros((n, cfg.n_out))
    fl = np.zeros(n, np.uint8)
    x0 = np.zeros((n, input_dim(cfg))) if want_x0 else None
    lib().orc_query(C.byref(cfg), _P(p, C.c_double), n, _P(pos, C.c_float),
                    _P(nrm, C.c_float), _P(ex, C.c_float), _P(al, C.c_float),
                    _P(mk, C.c_uint8), _P(E, C.c_double), _P(Lo, C.c_double),
                    _P(fl, C.c_uint8), _P(x0, C.c_double))
    if want_x0:
        return E, Lo, fl, x0
    return E, Lo, fl


def corners(cfg: Config, p):
    """Within-level corner indices [L, 8] and trilinear weights [L, 8]."""
    p = _f32(p).reshape(3)
    idx = np.zeros((cfg.n_levels, 8), np.int64)
    w = np.zeros((cfg.n_levels, 8))
    lib().orc_corners(C.byref(cfg), _P(p, C.c_float), _P(idx, C.c_int64), _P(w, C.c_double))
    return idx, w


def corners_many(cfg: Config, pos):
    """Within-level corner indices [n, L, 8] of n points (corners() per point)."""
    pos = _f32(pos).reshape(-1, 3)
    n = len(pos)
    idx = np.zeros((n, cfg.n_levels, 8), np.int64)
    lib().orc_corners_n(C.byref(cfg), _P(pos, C.c_float), n, _P(idx, C.c_int64))
    return idx


# ---------------------------------------------------------------- training
def loss_grad(cfg: Config, params, pos, nrm, target, extra=None, valid=None, eps=0.01):
    """Eq. 3 relative L2 loss and its exact gradient w.r.t. every parameter."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    pos = _f32(pos).reshape(-1, 3)
    nrm = _f32(nrm).reshape(-1, 3)
    tg = _f32(target).reshape(-1, cfg.n_out)
    n = pos.shape[0]
    ex = None if extra is None else _f32(extra).reshape(n, -1)
    vd = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    g = np.zeros(p.size)
    loss = lib().orc_loss_grad(C.byref(cfg), _P(p, C.c_double), n, _P(pos, C.c_float),
                               _P(nrm, C.c_float), _P(ex, C.c_float), _P(tg, C.c_float),
                               _P(vd, C.c_uint8), eps, _P(g, C.c_double))
    return float(loss), g


def loss(cfg: Config, params, pos, nrm, target, extra=None, valid=None, eps=0.01):
    p = np.ascontiguousarray(params, dtype=np.float64)
    pos = _f32(pos).reshape(-1, 3)
    nrm = _f32(nrm).reshape(-1, 3)
    tg = _f32(target).reshape(-1, cfg.n_out)
    n = pos.shape[0]
    ex = None if extra is None else _f32(extra).reshape(n, -1)
    vd = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    return float(lib().orc_loss(C.byref(cfg), _P(p, C.c_double), n, _P(pos, C.c_float),
                                _P(nrm, C.c_float), _P(ex, C.c_float), _P(tg, C.c_float),
                                _P(vd, C.c_uint8), eps))


def adam(params, grads, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """Kingma & Ba Adam, in place on float64 arrays (Sec. 4.5)."""
    for a in (params, grads, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(params.size, _P(params, C.c_double), _P(grads, C.c_double),
                   _P(m, C.c_double), _P(v, C.c_double), lr, beta1, beta2, eps, step)


def init_params(cfg: Config, seed, lo, hi):
    """Seeded initial parameters: grid uniform on [lo, hi), weights
    Xavier-uniform; parameter k from generator stream (seed, k, 0, 3)."""
    out = np.empty(n_params(cfg), dtype=np.float32)
    lib().orc_init_params(C.byref(cfg), int(seed), float(lo), float(hi), _P(out, C.c_float))
    return out


def lr_at(step, s1, s_end, lr0=1e-2, lr1=1e-4):
    """Sec. 4.5 schedule: lr0, then exponential decay to lr1."""
    return float(lib().orc_lr(step, s1, s_end, lr0, lr1))


# ---------------------------------------------------------------- random numbers
def philox4x64(ctr, key):
    c = (C.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) for x in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64(c, k, o)
    return [int(x) for x in o]


def uniform(seed, a, b, stream, dim):
    return float(lib().orc_uniform(seed, a, b, stream, dim))


# ---------------------------------------------------------------- Monte Carlo
def mc_irradiance(prims, x, nrm, spp, bounces, flags, seed, point_id=None, motion=None, t=None):
    """Eq. 1 indirect irradiance by Monte Carlo (Sec. 4.5 targets).  The
    random stream of point i is keyed by point_id[i] (default i).  A scene
    that changes with a scene variable (Sec. 6): primitive k translated by
    t[i] * motion[k] at point i.
    Returns (E [n,3], var [n,3], backfaces [n], valid [n])."""
    pr = np.ascontiguousarray(prims)
    x = _f32(x).reshape(-1, 3)
    nrm = _f32(nrm).reshape(-1, 3)
    n = x.shape[0]
    E = np.zeros((n, 3))
    var = np.zeros((n, 3))
    bf = np.zeros(n, np.int32)
    vd = np.zeros(n, np.uint8)
    ids = None
    if point_id is not None:
        ids = np.ascontiguousarray(point_id, dtype=np.uint64).reshape(-1)
        assert ids.size == n
    mo = None if motion is None else _f32(motion).reshape(len(pr), 3)
    tv = None if t is None else _f32(t).reshape(n)
    lib().orc_mc_irradiance(pr.ctypes.data, len(pr), _P(x, C.c_float), _P(nrm, C.c_float),
                            None if ids is None else ids.ctypes.data, n, int(spp), int(bounces), int(flags), int(seed),
                            _P(E, C.c_double), _P(var, C.c_double),
                            _P(bf, C.c_int32), _P(vd, C.c_uint8), _P(mo, C.c_float),
                            _P(tv, C.c_float))
    return E, var, bf, vd


def dynamic_ao(tris, pos, nrm, rays, radius, eps, seed, point_id=None):
    """Dynamic ambient occlusion (Sec. 4.4): visibility of the hemisphere of
    each point against the dynamic triangles [m,3,3] within `radius`, from
    `rays` cosine-distributed directions of the point's stream (keyed by
    point_id[i], default i).  Returns [n] visibilities in [0, 1]."""
    tr = _f32(tris).reshape(-1, 9)
    pos = _f32(pos).reshape(-1, 3)
    nrm = _f32(nrm).reshape(-1, 3)
    n = pos.shape[0]
    ids = None
    if point_id is not None:
        ids = np.ascontiguousarray(point_id, dtype=np.uint64).reshape(-1)
        assert ids.size == n
    vis = np.zeros(n)
    lib().orc_dynamic_ao(_P(tr, C.c_float), tr.shape[0], _P(pos, C.c_float), _P(nrm, C.c_float),
                         None if ids is None else ids.ctypes.data, n, int(rays), float(radius),
                         float(eps), int(seed), _P(vis, C.c_double))
    return vis


def sample_points(prims, lo, hi, count, n_surface, seed, with_t=False):
    """Sec. 4.5 training points: volume points then surface points (and a
    scene variable per point, uniform on [0, 1), with with_t)."""
    pr = np.ascontiguousarray(prims)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    x = np.zeros((count, 3), np.float32)
    n = np.zeros((count, 3), np.float32)
    t = np.zeros(count, np.float32) if with_t else None
    lib().orc_sample_points(pr.ctypes.data, len(pr), _P(lo, C.c_double), _P(hi, C.c_double),
                            int(count), int(n_surface), int(seed), _P(x, C.c_float),
                            _P(n, C.c_float), _P(t, C.c_float))
    return (x, n, t) if with_t else (x, n)


def upsample(cfg: Config, width, height, pos, nrm, half_E, mask=None, albedo=None,
             sigma_px=1.0, sigma_pos=0.1, normal_power=8):
    """Half-resolution rendering (Sec. 4.4): joint bilateral upsampling of
    the irradiance at pixels (2x, 2y) to every pixel, then Eq. 2.
    Returns (E [H*W, 3], L [H*W, 3], flags [H*W] uint8)."""
    n = width * height
    pos = _f32(pos).reshape(n, 3)
    nrm = _f32(nrm).reshape(n, 3)
    hw, hh = (width + 1) // 2, (height + 1) // 2
    hE = np.ascontiguousarray(half_E, dtype=np.float64).reshape(hh * hw, 3)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(n)
    al = None if albedo is None else _f32(albedo).reshape(n, 3)
    E = np.zeros((n, 3))
    Lo = np.zeros((n, 3))
    fl = np.zeros(n, np.uint8)
    lib().orc_upsample(C.byref(cfg), int(width), int(height), _P(pos, C.c_float),
                       _P(nrm, C.c_float), _P(mk, C.c_uint8), _P(al, C.c_float),
                       _P(hE, C.c_double), float(sigma_px), float(sigma_pos), int(normal_power),
                       _P(E, C.c_double), _P(Lo, C.c_double), _P(fl, C.c_uint8))
    return E, Lo, fl


def half_samples(width, height, *arrays):
    """The pixels (2x, 2y) of full-resolution [H*W, ...] arrays, row-major."""
    out = []
    for a in arrays:
        a = np.asarray(a)
        b = a.reshape((height, width) + a.shape[1:])[::2, ::2]
        out.append(np.ascontiguousarray(b.reshape((-1,) + a.shape[1:])))
    return out


def config_from_workload(w) -> Config:
    return make_config(**w.model_dict())
