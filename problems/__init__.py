"""Seeded synthetic inputs for sequences of sparse SPD systems.

This package only manufactures inputs (matrices, right-hand sides, random
fields).  It contains none of the solver's arithmetic: no Krylov iteration,
no projection, no POD.  Both the CPU oracle and the GPU library consume what
it produces, so the two sides always see bit-identical inputs.
"""

from .grf import FourierField
from .fv import FVDiffusion
from .configs import (
    Config1Diffusion2D,
    Config2Diffusion3D,
    Config3Elasticity,
    Config4Batch,
    Config4Member,
    Config5Adjoint,
    config1,
    config2,
    config3,
    config4,
    config5,
)
from .elasticity import Q1Elasticity
from . import tiny

__all__ = [
    "FourierField",
    "FVDiffusion",
    "Config1Diffusion2D",
    "Config2Diffusion3D",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "Config3Elasticity",
    "Config4Batch",
    "Config4Member",
    "Config5Adjoint",
    "Q1Elasticity",
    "tiny",
]
