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

Medium variants change the projected area, NDF and proposal terms:
  anisotropic kernel   projected area +12 (cosine to the normal, scaled spread), NDF +20
  GGX macrofacet       projected area +5, NDF -20, phase sampling -35 (closed-form GGX
                       visible normals instead of the Newton slope inversion), mixture pdf -10
  conductor Fresnel    +30 per phase evaluation and per sampling weight (two square roots,
                       two divisions)

A GP conditioned on n observations adds, per point evaluation, the posterior of value and
gradient: per observation the kernel value, the mean and mean-gradient terms (20) and the
per-row closing of the triangular solve (29), 8 per entry of the lower triangle of the
inverse Cholesky factor (n (n + 1) / 2 entries), and the gradient covariance given f = 0
with its 3x3 Cholesky factor (55); its projected area (+12) and NDF (+30, two 3x3
triangular solves) cost a little more than the isotropic forms.
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


COND_PER_OBS = 20 + 29
COND_PER_PAIR = 8
COND_BASE = 55
COND_PROJ = 12
COND_NDF = 30


def n_observations(scene) -> int:
    obs = getattr(scene, "observations", None)
    return 0 if obs is None else int(len(obs))


def point_flops(scene) -> int:
    f = POINT_BASE
    n = n_observations(scene)
    if n:
        f += COND_BASE + COND_PER_OBS * n + COND_PER_PAIR * n * (n + 1) // 2
    if scene.mean_kind == 1:
        import numpy as np
        kinds = np.asarray(scene.prims)[:, 0]
        f += int((kinds == 0).sum()) * SPHERE_SDF + int((kinds == 1).sum()) * BOX_SDF
    if scene.offset_grid is not None:
        f += OFFSET_GRID
    if scene.variance_grid is not None:
        f += VARIANCE_GRID
    return f


ANISO_PROJ, ANISO_NDF = 12, 20
GGX_PROJ, GGX_NDF, GGX_SAMPLE, GGX_PDF = 5, -20, -35, -10
FRESNEL = 30


def per_event(scene) -> dict:
    p = point_flops(scene)
    cp, cn = (COND_PROJ, COND_NDF) if n_observations(scene) else (0, 0)
    ln = float(getattr(scene, "lengthscale_n", 0.0))
    if ln > 0.0 and ln != float(scene.lengthscale):
        cp, cn = cp + ANISO_PROJ, cn + ANISO_NDF
    sample = 0
    if int(getattr(scene, "ndf_kind", 0)) == 1:
        cp, cn, sample = cp + GGX_PROJ, cn + GGX_NDF, GGX_SAMPLE + GGX_PDF
    fr = FRESNEL if float(getattr(scene, "fresnel_eta", 0.0)) > 0.0 else 0
    return {
        "track_steps": TRACK_EXTRA + p + DENSITY + PROJ + cp,
        "nee_steps": NEE_EXTRA + p + DENSITY + PROJ + cp,
        "cells": CELL,
        "phase": REAL + p + cp + cn + sample + fr,
        "nee": NEE + cn + fr,
    }


def flops_from_counters(scene, counters: dict) -> float:
    pe = per_event(scene)
    return float(sum(pe[k] * counters.get(k, 0) for k in pe))
