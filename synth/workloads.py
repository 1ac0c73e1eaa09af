"""Named synthetic workloads shaped like the paper's scatterers.

Each entry returns a dict with the grid(s), permittivity map(s), incidence
angles and the solver settings that go with the workload.  Nothing here is
read from disk; everything is generated from the stated seeds.
"""

from __future__ import annotations

import math

from .objects import (
    centred_grid,
    cylinder,
    square,
    layered_square,
    random_field_object,
    inclusion_object,
    sinusoid_object,
)


def _cyl_small():
    # radius 0.5 lambda, eps 4, in a 1.2 lambda square of 64 x 64 cells; P = 128^2
    g = centred_grid(64, 1.2)
    return dict(name="cyl64_eps4", grids=[g], eps=[cylinder(g, 0.5, 4.0 + 0j)], psi=[0.0],
                restart=20, regularize=False, deflate_k=0, radius=0.5, eps_obj=4.0 + 0j)


def _cyl_hard():
    # radius 2 lambda, eps -2.5+0.2i, 256 x 256 cells over 4.4 lambda, incidence 30 degrees
    g = centred_grid(256, 4.4)
    return dict(name="cyl256_eps-2.5+0.2i", grids=[g], eps=[cylinder(g, 2.0, -2.5 + 0.2j)],
                psi=[math.pi / 6.0], restart=30, regularize=True, deflate_k=20,
                radius=2.0, eps_obj=-2.5 + 0.2j)


def _batched(sizes=(128, 256, 512, 1024), per_size=4, n_angles=64):
    grids, eps = [], []
    o = 0
    for n in sizes:
        for _ in range(per_size):
            g, e = random_field_object(n, seed=1000 + o)
            grids.append(g)
            eps.append(e)
            o += 1
    psi = [2.0 * math.pi * j / n_angles for j in range(n_angles)]
    return dict(name="randfield_batched", grids=grids, eps=eps, psi=psi, restart=30,
                regularize=False, deflate_k=16)


def _stress(n=2048, side=25.6):
    g, e = inclusion_object(n=n, side=side)
    return dict(name="ellipse_inclusions_2048", grids=[g], eps=[e],
                psi=[2.0 * math.pi * j / 8 for j in range(8)], restart=40, regularize=True,
                deflate_k=40)


def _paper_squares(nodes=61):
    # the three square scatterers of the paper's TE table: side = lambda, h = lambda/(nodes-1)
    side = 1.0
    g = centred_grid(nodes, side * nodes / (nodes - 1))
    return dict(name="paper_squares", grids=[g, g, g],
                eps=[square(g, side, 16.0 + 0j), square(g, side, -16 + 1.5j),
                     layered_square(g, side, 16.0 + 0j, 2.5 + 20j)],
                psi=[0.0], restart=40, regularize=True, deflate_k=14)


def _paper_sinusoid(nodes=233, side=4.0):
    # nodes spanning the object: cell centres from -a/2 to a/2 with a = side
    g, e = sinusoid_object(nodes, side * nodes / (nodes - 1), a=side)
    return dict(name="paper_sinusoid", grids=[g], eps=[e], psi=[0.0], restart=1440,
                regularize=True, deflate_k=180)


WORKLOADS = {
    "cyl_small": _cyl_small,
    "cyl_hard": _cyl_hard,
    "batched": _batched,
    "stress": _stress,
    "paper_squares": _paper_squares,
    "paper_sinusoid": _paper_sinusoid,
}


def workload(name: str, **kw) -> dict:
    return WORKLOADS[name](**kw)
