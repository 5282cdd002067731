"""Seeded synthetic scene generators shared by the oracle tests and the GPU path.

This package only draws random fields and lays out the inputs (emissivity,
opacity, line parameters, velocities, directions, ray samples).  It holds none
of the formal-solution arithmetic: no profile evaluation, no mip chain, no
traversal, no radiative-transfer update.
"""
from .scenes import (  # noqa: F401
    C_KMS,
    grf,
    directions_2d,
    directions_fibonacci,
    make_cfg1,
    make_cfg2,
    make_cfg3,
    make_cfg4_scene,
    make_prominence,
    cfg4_specs,
)
