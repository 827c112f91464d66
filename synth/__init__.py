"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the
benchmark.  Random numbers and array layout only; no part of the method."""
from .scenes import (WORKSPACE, ROOM, Workload, workload, uniform_cube_cloud,
                     uniform_spheres, tabletop_cloud, room_cloud, depth_frame, chain_template,
                     posed_spheres, pose_edges)

__all__ = ["WORKSPACE", "ROOM", "Workload", "workload", "uniform_cube_cloud",
           "uniform_spheres", "tabletop_cloud", "room_cloud", "depth_frame", "chain_template",
           "posed_spheres", "pose_edges"]
