"""Seeded synthetic inputs for the Neural Irradiance Volume hot path.

This package only draws random numbers and builds input data: query points,
model parameter values, rooms made of boxes and rectangles, and G-buffers made
by casting primary rays into those rooms (primary visibility is outside the
method and outside its timings, Sec. 5.2 and App. F).  It holds none of the
method's arithmetic: no encoding, no network, no irradiance estimation.  Both
the CPU oracle and the GPU library consume what it produces.
"""
from .workloads import WORKLOADS, Workload, get_workload
from .params import make_params, xavier_bound
from .scene import (PRIM_DTYPE, PRIM_BOX, PRIM_RECT, PRIM_DISK, make_room,
                    room_prims, enclosure_prims, disk_prim, rect_prim, box_prim,
                    scene_bounds, room_motion)
from .gbuffer import (Camera, default_camera, cast_gbuffer, make_room_gbuffer,
                      make_workload_gbuffer, workload_meshes, mesh_triangles)
from .mesh import icosphere, displaced_sphere
from .points import unit_cube_queries, uniform_unit_normals
from .batch import make_room_gbuffers

__all__ = [
    "WORKLOADS", "Workload", "get_workload", "make_params", "xavier_bound",
    "PRIM_DTYPE", "PRIM_BOX", "PRIM_RECT", "PRIM_DISK", "make_room", "room_prims",
    "enclosure_prims", "disk_prim", "rect_prim", "box_prim", "scene_bounds",
    "Camera", "default_camera", "cast_gbuffer", "make_room_gbuffer",
    "unit_cube_queries", "uniform_unit_normals", "make_room_gbuffers",
    "make_workload_gbuffer", "icosphere", "displaced_sphere", "room_motion",
    "workload_meshes", "mesh_triangles",
]
