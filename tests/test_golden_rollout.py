"""The script that writes the stored 100-step oracle rollout evaluates each
right-hand side of the periodic box in z-slabs with one halo element on each
side.  This pins that evaluation: on a mesh with unequal element widths in
every direction it must reproduce the oracle's whole-mesh right-hand side
bit for bit, for any slab thickness (including a ragged last slab)."""

import importlib.util
import os

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs
from oracle.mesh import Mesh
from oracle.physics import Gas

from _cases import random_faces, random_state

HERE = os.path.dirname(os.path.abspath(__file__))


def _script():
    spec = importlib.util.spec_from_file_location(
        "make_tgv_n7_rollout", os.path.join(HERE, "golden", "make_tgv_n7_rollout.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("slab", [1, 2, 3, 7])
def test_slab_rhs_is_the_whole_mesh_rhs(slab):
    mk = _script()
    rng = np.random.default_rng(7)
    faces = (random_faces(4, 0.0, 2.0, rng), random_faces(3, 0.0, 3.0, rng),
             random_faces(7, 0.0, 4.0, rng))
    mesh = Mesh(3, faces)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=0.01, Pr=0.72)
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=1.0 / (1.4 * 0.01), p_amp=0.05)
    ref = rhs(U, mesh, g)
    got = mk.slab_rhs(U, mesh, g, slab)
    assert torch.equal(got, ref)


def test_samples_fixed_and_distinct():
    s = _script().sample_elements(32 ** 3)
    assert s.size == 64 and np.unique(s).size == 64
    assert s.min() >= 0 and s.max() < 32 ** 3
    assert s[0] == 0 and s[1] == 31 + 32 * (17 + 32 * 5)
