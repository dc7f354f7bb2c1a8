"""The synthetic workloads, named by what they are.

Model hyper-parameters follow Sec. 4.1 (hash table size, latent size, level
scale and coarsest resolution) where a workload does not fix them; the network
is a stack of ReLU layers with a linear RGB output (Sec. 4.1).
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple
import math

ROOM_LO = (0.0, 0.0, 0.0)
ROOM_HI = (10.0, 4.0, 10.0)


@dataclass(frozen=True)
class Workload:
    name: str
    # model
    n_levels: int
    log2_T: int
    n_features: int
    base_res: float
    per_level_scale: float
    sh_bands: int
    n_extra: int
    extra_bands: int
    width: int
    n_hidden: int
    n_out: int
    aabb_min: Tuple[float, float, float]
    aabb_max: Tuple[float, float, float]
    grid_init: Tuple[float, float]
    # workload
    frames: Tuple[Tuple[int, int], ...] = ()
    n_queries: int = 0
    scene_seeds: Tuple[int, ...] = ()
    param_seed: int = 0
    point_seed: int = 0
    precision: str = "fp16"
    extra_values: Tuple[float, ...] = ()
    meshes: Tuple[Tuple[int, Tuple[float, float, float]], ...] = ()  # (seed, centre)
    pos_bands: int = 0   # positional code of x (models without grid levels)
    notes: str = ""

    def model_dict(self):
        return dict(n_levels=self.n_levels, log2_T=self.log2_T,
                    n_features=self.n_features, base_res=self.base_res,
                    per_level_scale=self.per_level_scale, sh_bands=self.sh_bands,
                    n_extra=self.n_extra, extra_bands=self.extra_bands,
                    width=self.width, n_hidden=self.n_hidden, n_out=self.n_out,
                    aabb_min=self.aabb_min, aabb_max=self.aabb_max,
                    pos_bands=self.pos_bands)


WORKLOADS = {
    # 128x128 queries in the unit cube, small hash grid; the parity workload.
    "unit_cube_16k": Workload(
        name="unit_cube_16k", n_levels=8, log2_T=14, n_features=2, base_res=4.0,
        per_level_scale=1.5, sh_bands=4, n_extra=0, extra_bands=0, width=64,
        n_hidden=2, n_out=3, aabb_min=(0.0, 0.0, 0.0), aabb_max=(1.0, 1.0, 1.0),
        grid_init=(-0.5, 0.5), n_queries=128 * 128, param_seed=1002,
        point_seed=1001, precision="fp32"),
    # one full-HD G-buffer of a 10x4x10 m room with 32 boxes; the query workload.
    "room_1080p": Workload(
        name="room_1080p", n_levels=16, log2_T=17, n_features=2, base_res=16.0,
        per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=0, extra_bands=0,
        width=64, n_hidden=3, n_out=3, aabb_min=ROOM_LO, aabb_max=ROOM_HI,
        grid_init=(-0.5, 0.5), frames=((1920, 1080),), scene_seeds=(2001,),
        param_seed=2002, precision="fp16"),
    # on-GPU training in the same room lit by two ceiling rectangles.
    "room_train": Workload(
        name="room_train", n_levels=16, log2_T=17, n_features=2, base_res=16.0,
        per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=0, extra_bands=0,
        width=64, n_hidden=3, n_out=3, aabb_min=ROOM_LO, aabb_max=ROOM_HI,
        grid_init=(-1e-4, 1e-4), n_queries=1 << 18, scene_seeds=(2001,),
        param_seed=3002, point_seed=3001, precision="fp16"),
    # eight G-buffers of uneven size over eight rooms, one launch.
    "batched_8_rooms": Workload(
        name="batched_8_rooms", n_levels=16, log2_T=17, n_features=2,
        base_res=16.0, per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=0,
        extra_bands=0, width=64, n_hidden=3, n_out=3, aabb_min=ROOM_LO,
        aabb_max=ROOM_HI, grid_init=(-0.5, 0.5),
        frames=((1280, 720), (1366, 768), (1600, 900), (1792, 1008),
                (1920, 1080), (2048, 1152), (2304, 1296), (2560, 1440)),
        scene_seeds=tuple(range(4000, 4008)), param_seed=4100, precision="fp16"),
    # a 4K G-buffer with a per-frame scene variable (6-D field), wider network.
    "room_4k_6d": Workload(
        name="room_4k_6d", n_levels=16, log2_T=19, n_features=2, base_res=16.0,
        per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=1, extra_bands=8,
        width=128, n_hidden=4, n_out=3, aabb_min=ROOM_LO, aabb_max=ROOM_HI,
        grid_init=(-0.5, 0.5), frames=((3840, 2160),), scene_seeds=(5001,),
        param_seed=5002, precision="bf16", extra_values=(0.0, 0.37, 1.0),
        meshes=((5101, (3.6, 1.3, 5.0)), (5102, (6.6, 1.7, 6.5)))),
}

# The room G-buffer under the grid-free models of Table 1: no grid levels, an
# eight-band positional code of x, a four-layer network of width 16, 32 or 64
# (Sec. 4.1).
for _w in (16, 32, 64):
    WORKLOADS[f"room_1080p_pe{_w}"] = Workload(
        name=f"room_1080p_pe{_w}", n_levels=0, log2_T=17, n_features=2, base_res=16.0,
        per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=0, extra_bands=0,
        width=_w, n_hidden=3, n_out=3, aabb_min=ROOM_LO, aabb_max=ROOM_HI,
        grid_init=(0.0, 0.0), frames=((1920, 1080),), scene_seeds=(2001,),
        param_seed=2002 + _w, precision="fp16", pos_bands=8)


# The room G-buffer under the grid networks of Table 1: 2, 4, 6 or 8 levels
# of four features (Sec. 4.1: T = 2^17, coarsest side 16, scale sqrt(2)), a
# four-layer network of width 64.
for _l in (2, 4, 6, 8):
    WORKLOADS[f"room_1080p_g{_l}"] = Workload(
        name=f"room_1080p_g{_l}", n_levels=_l, log2_T=17, n_features=4, base_res=16.0,
        per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=0, extra_bands=0,
        width=64, n_hidden=3, n_out=3, aabb_min=ROOM_LO, aabb_max=ROOM_HI,
        grid_init=(-0.5, 0.5), frames=((1920, 1080),), scene_seeds=(2001,),
        param_seed=2100 + _l, precision="fp16")


# On-GPU training of the field with one scene variable (Sec. 6): the room of
# room_train with its two ceiling lights sliding along x and one box moving
# along z as t goes from 0 to 1 (niv_synth.scene.room_motion); the hash
# table doubled as the paper does for this application.
WORKLOADS["room_train_6d"] = Workload(
    name="room_train_6d", n_levels=16, log2_T=18, n_features=2, base_res=16.0,
    per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=1, extra_bands=8, width=64,
    n_hidden=3, n_out=3, aabb_min=ROOM_LO, aabb_max=ROOM_HI, grid_init=(-1e-4, 1e-4),
    n_queries=1 << 18, scene_seeds=(2001,), param_seed=6002, point_seed=6001,
    precision="fp16", extra_values=(0.0, 0.5, 1.0))


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]
