"""Pins of the oracle's inverse mapping (Sec. II-B, Eq. (4)).

q_a = sum_i q_i f_ai / S_a with the pair weights of the forward mapping.  The
pins do not retype that sum: a particle beside one wall of two boxes takes the
two box values in the proportions of the kernel mass on each side of the wall
(the half-space integral, by nested quadrature); a particle alone in a cell
takes the cell's value; a constant field maps to itself; and the mapped
quantity's mass is conserved, sum_a m_a q_a = sum_i q_i M_i.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import Cells
from tests.test_oracle_pins import box_cell, half_space


def two_boxes():
    """Cells [0, 0.5] x [0, 1]^2 and [0.5, 1] x [0, 1]^2 (faces counter-clockwise from outside)."""
    a = box_cell((0.0, 0.0, 0.0), (0.5, 1.0, 1.0))
    b = box_cell((0.5, 0.0, 0.0), (1.0, 1.0, 1.0))
    verts = np.vstack([a.verts, b.verts])
    fvert = np.concatenate([a.face_vert, b.face_vert + len(a.verts)]).astype(np.int32)
    fvo = np.concatenate([a.face_vert_off, b.face_vert_off[1:] + a.face_vert_off[-1]]).astype(np.int64)
    plane = np.vstack([a.face_plane, b.face_plane])
    nb = np.concatenate([a.face_nb, b.face_nb])
    return Cells(np.array([0, 6, 12], dtype=np.int64), fvo, fvert, plane, nb, verts,
                 np.array([0.5, 0.5]), (0.0, 0.0, 0.0, 1.0, 1.0, 1.0))


@pytest.mark.parametrize("u", [0.0, 0.3, 0.77, 1.0, 1.4, 1.95])
def test_particle_beside_a_wall_takes_both_sides(u):
    h = 0.1
    c = two_boxes()
    p = synth.Particles(np.array([[0.5 - u * h, 0.5, 0.5]]), np.array([1.0]), np.array([h]))
    o = oracle.map_particles(p, c)
    q = np.array([2.0, 7.0])
    qa = oracle.map_back(q, o, 1)[0]
    beyond = half_space(u)  # kernel mass past the wall, in the right box
    assert qa == pytest.approx(q[0] * (1.0 - beyond) + q[1] * beyond, rel=1e-12, abs=1e-13)


def test_particle_alone_in_a_cell_takes_its_value():
    c = box_cell((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    p = synth.Particles(np.array([[0.4, 0.55, 0.5]]), np.array([1.0]), np.array([0.15]))
    o = oracle.map_particles(p, c)
    assert oracle.map_back(np.array([-3.25]), o, 1)[0] == pytest.approx(-3.25, rel=1e-14)


def test_constant_field_maps_to_itself():
    p, c = synth.workload("clumps", 600, 61)
    o = oracle.map_particles(p, c)
    qa = oracle.map_back(np.full(c.n_cells, 3.7), o, p.n)
    touching = o["S"] > 0
    assert touching.all()
    assert np.abs(qa - 3.7).max() < 1e-13


def test_mapped_mass_is_conserved():
    p, c = synth.workload("uniform", 512, 62)
    o = oracle.map_particles(p, c)
    q = np.random.default_rng(5).uniform(-1.0, 2.0, c.n_cells)
    qa = oracle.map_back(q, o, p.n)
    lhs = float(np.dot(p.m, qa))
    rhs = float(np.dot(q, o["M"]))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    # a transposed pairing (cell values read at particle indices) breaks it
    bad = {"pair_p": o["pair_c"], "pair_c": o["pair_p"], "f": o["f"], "S": np.ones(c.n_cells)}
    assert abs(float(np.dot(p.m, oracle.map_back(q, bad, p.n))) - rhs) > 1e-6
