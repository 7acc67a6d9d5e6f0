"""Seeded synthetic porous images and pore labels.

This package only draws inputs: binary voxel images of grain packings and a
watershed labelling of their void space.  It holds none of the solver's
arithmetic (no discretisation, no decomposition rule, no preconditioner), so
both the FP64 oracle and the HIP library can consume what it produces.

The paper decomposes its images with a watershed of the distance map
(Section 3.2.1, primary grids); its own images (PD4, GLD4, Berea, Granular)
are not available, so random disk / sphere packings of similar structure stand
in for them.
"""
from .packing import disk_packing_rsa, boolean_packing, channel
from .watershed import watershed_labels, throat_labels
from .workloads import make_workload, make_batch, WORKLOADS

__all__ = ["disk_packing_rsa", "boolean_packing", "channel",
           "watershed_labels", "throat_labels", "make_workload", "make_batch", "WORKLOADS"]
