"""Algorithmic work model of the forward tracer (used for roofline reporting).

Floating-point operations are counted from the arithmetic each event performs as
written in the tracer: an add, multiply, compare-free min/max or division counts 1, a
fused multiply-add 2, and every special function (exp, log, sqrt, erfc, erfcx, erfinv,
sin/cos) counts 1.  Double-precision ray bookkeeping is counted like single precision.
Integer work (Philox rounds, cell indices) is not counted.

Per-event counts:
  TRACK_STEP  tentative collision of delta tracking: distance update (3), position (6),
              accept test (2), point statistics (mean geometry, grids), density (5),
              projected area (20), extinction product (1)
  NEE_STEP    tentative collision of ratio tracking: as above with the transmittance
              update (3) in place of the accept test
  CELL        majorant-cell crossing: three boundary distances (12), optical-depth
              update (2), axis selection (2)
  PHASE       real collision with phase sampling: proposal frame (30), Beckmann slope
              inversion (about five Newton steps of 15), slope to normal (15), mixture
              pdf (30), NDF (35), projected area (20), weight (5), reflection (15)
  NEE         light connection: light direction and box clip (32), phase evaluation (70)
"""

# point statistics cost by mean kind: sphere SDF per primitive, box SDF per primitive,
# plane, constant; trilinear grids with gradient (offset) and value only (variance)
SPHERE_SDF = 14
BOX_SDF = 25
PLANE = 0
OFFSET_GRID = 40
VARIANCE_GRID = 22
POINT_BASE = 2          # sigma = sqrt(var), s = sigma / l

DENSITY = 5
PROJ = 20
TRACK_EXTRA = 3 + 6 + 2 + 1
NEE_EXTRA = 3 + 6 + 3 + 1
CELL = 16
REAL = 30 + 75 + 15 + 30 + 35 + 20 + 5 + 15
NEE = 32 + 70


def point_flops(scene) -> int:
    f = POINT_BASE
    if scene.mean_kind == 1:
        import numpy as np
        kinds = np.asarray(scene.prims)[:, 0]
        f += int((kinds == 0).sum()) * SPHERE_SDF + int((kinds == 1).sum()) * BOX_SDF
    if scene.offset_grid is not None:
        f += OFFSET_GRID
    if scene.variance_grid is not None:
        f += VARIANCE_GRID
    return f


def per_event(scene) -> dict:
    p = point_flops(scene)
    return {
        "track_steps": TRACK_EXTRA + p + DENSITY + PROJ,
        "nee_steps": NEE_EXTRA + p + DENSITY + PROJ,
        "cells": CELL,
        "phase": REAL + p,
        "nee": NEE,
    }


def flops_from_counters(scene, counters: dict) -> float:
    pe = per_event(scene)
    return float(sum(pe[k] * counters.get(k, 0) for k in pe))
