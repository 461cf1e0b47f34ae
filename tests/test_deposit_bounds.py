"""The facts the GPU current deposit relies on, checked on the host in FP64
over random moves and the edge cases (Esirkepov's decomposition with the
cloud-in-cell shape, Comput. Phys. Commun. 135, 144, 2001):

- a move of less than one cell puts the old and new shapes on three
  consecutive nodes, starting one node below the old cell when the new
  position is below it and at the old cell otherwise (the stencil loops run
  over those three nodes);
- the change D = S1 - S0 sums to zero, so the last partial sum along a
  component's own axis vanishes and is not stored;
- every partial sum of D is bounded by the move in cells, and the transverse
  factors lie in [0, 1], so a contribution is bounded by |c_a| |du_a| (the
  scale of the deposit's fixed-point LDS sums)."""
import numpy as np
import pytest


def _cic(r):
    """CIC weights of a particle at r cells from node i on nodes i-1 .. i+2."""
    c = np.arange(4) - 1.0
    return np.maximum(0.0, 1.0 - np.abs(r[..., None] - c))


def _moves(n, rng):
    f0 = rng.uniform(0.0, 1.0, n)
    du = rng.uniform(-1.0, 1.0, n)
    # edge cases: at a node, moves that end exactly on a node, near-cell moves
    f0[:6] = [0.0, 0.0, 0.5, 0.999999, 0.25, 0.0]
    du[:6] = [0.0, -0.999999, -0.5, 0.000001, 0.75, 0.999999]
    return f0, du


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_three_node_window_holds_both_shapes(seed):
    rng = np.random.default_rng(seed)
    f0, du = _moves(200000, rng)
    r1 = f0 + du
    s0, s1 = _cic(f0), _cic(r1)
    o = np.where(r1 < 0.0, 0, 1)
    outside = np.where(o[:, None] == 0, np.array([0, 0, 0, 1]), np.array([1, 0, 0, 0]))
    assert np.all(s0 * outside == 0.0)
    assert np.all(s1 * outside == 0.0)
    # the shapes are partitions of unity
    np.testing.assert_allclose(s0.sum(1), 1.0, atol=1e-14)
    np.testing.assert_allclose(s1.sum(1), 1.0, atol=1e-14)


@pytest.mark.parametrize("seed", [4, 5])
def test_partial_sums_of_the_change_are_bounded_by_the_move(seed):
    rng = np.random.default_rng(seed)
    f0, du = _moves(200000, rng)
    d = _cic(f0 + du) - _cic(f0)
    part = np.cumsum(d, axis=1)
    np.testing.assert_allclose(part[:, -1], 0.0, atol=1e-14)
    assert np.all(np.abs(part) <= np.abs(du)[:, None] + 1e-14)
    # and it is tight: some moves reach it
    nz = np.abs(du) > 1e-3
    assert (np.abs(part).max(1)[nz] / np.abs(du)[nz]).max() > 0.999


@pytest.mark.parametrize("seed", [6, 7])
def test_transverse_factors_lie_in_the_unit_interval(seed):
    rng = np.random.default_rng(seed)
    fy, duy = _moves(100000, rng)
    fz, duz = _moves(100000, rng)
    s0y, s0z = _cic(fy), _cic(fz)
    dy, dz = _cic(fy + duy) - s0y, _cic(fz + duz) - s0z
    # 3D: the path average of the product of the two transverse shapes
    f3 = (s0y[:, :, None] * s0z[:, None, :] + 0.5 * dy[:, :, None] * s0z[:, None, :]
          + 0.5 * s0y[:, :, None] * dz[:, None, :] + dy[:, :, None] * dz[:, None, :] / 3.0)
    assert f3.min() >= -1e-15 and f3.max() <= 1.0 + 1e-15
    # it sums to one over the transverse nodes (the current's total is q w v)
    np.testing.assert_allclose(f3.sum((1, 2)), 1.0, atol=1e-13)
    # 2D: the path average of one transverse shape
    f2 = s0y + 0.5 * dy
    assert f2.min() >= -1e-15 and f2.max() <= 1.0 + 1e-15
