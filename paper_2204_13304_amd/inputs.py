"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and fills arrays; it holds none of the
solver arithmetic (no operator application, no sweep).  Right-hand sides of
the form b = A*1 are formed by whichever side consumes them.

All draws use numpy.random.default_rng(seed) in C order, so the oracle and
the GPU path see bit-identical inputs.

Workload recipes (HPCG- and NPB-LU-shaped synthetic stand-ins; the paper
uses no dataset):
  const27 small:   16^3 grid, b = A*1, x0 = 0
  const27 mg:      104^3 / 256^3, b = A*1 + N(0, 1e-3) with seeds 2 / 3
  block7 ssor:     162^3 x 5, blocks U(-1,1) seed 4, centre block + 10*I
  var7 adjoint:    128^3 (seed 5) and 16^3 (seed 55): face coefficients
                   exp(N(0, 0.5^2)) drawn kx, ky, kz, then f ~ N(0,1), then
                   the target u_t ~ N(0,1)
"""
from __future__ import annotations

import numpy as np


def grid_shape(n, m=None, p=None):
    """(nz, ny, nx) for an n x m x p grid (x fastest); cube if m, p omitted."""
    nx = n
    ny = n if m is None else m
    nz = n if p is None else p
    return (nz, ny, nx)


def normal(seed, shape, std=1.0, mean=0.0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.normal(mean, std, size=shape).astype(dtype, copy=False)


def standard_normal(seed, shape, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=shape).astype(dtype, copy=False)


def uniform(seed, shape, lo=-1.0, hi=1.0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(dtype, copy=False)


def rhs_perturbation(seed, shape, std=1e-3):
    """The N(0, std^2) perturbation added to b = A*1 in the MG-PCG runs."""
    return normal(seed, shape, std=std)


def block7_blocks(seed=4, dominance=10.0):
    """Seven 5x5 blocks (centre, -x, +x, -y, +y, -z, +z), entries U(-1, 1);
    the centre block gets +dominance on its diagonal."""
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, size=(7, 5, 5))
    b[0] += dominance * np.eye(5)
    return np.ascontiguousarray(b)


def bt_problem(seed, shape, dominance=20.0):
    """Blocks and right-hand side of 5x5 block-tridiagonal line systems on a
    grid of shape (nz, ny, nx): per point the blocks A, B, C with entries
    U(-1, 1), shape (3, nz, ny, nx, 5, 5), B getting +dominance on its
    diagonal; r ~ N(0, 1) of shape (nz, ny, nx, 5)."""
    rng = np.random.default_rng(seed)
    coef = rng.uniform(-1.0, 1.0, size=(3,) + tuple(shape) + (5, 5))
    coef[1] += dominance * np.eye(5)
    r = rng.standard_normal(tuple(shape) + (5,))
    return np.ascontiguousarray(coef), r


def var7_problem(seed, shape, log_std=0.5):
    """Face coefficients and data for the variable-coefficient diffusion
    problem on a grid of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    kx = np.exp(rng.normal(0.0, log_std, size=(nz, ny, nx + 1)))
    ky = np.exp(rng.normal(0.0, log_std, size=(nz, ny + 1, nx)))
    kz = np.exp(rng.normal(0.0, log_std, size=(nz + 1, ny, nx)))
    f = rng.standard_normal(size=shape)
    u_t = rng.standard_normal(size=shape)
    return dict(kx=kx, ky=ky, kz=kz, f=f, u_t=u_t)
