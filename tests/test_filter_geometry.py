"""Host checks of the geometric facts the crowded-cell near-list filter
relies on (no GPU): on a grid of at least four cells per axis, whose cell
edge is at least the contact reach R_i + R_j + 2 c_m (Alg. 1's cell size
2.5 R'max + 2.5 c_m bounds it), a candidate shifted once to the periodic
image nearest a cell's centre differs from every particle of that cell by
exactly the minimum image whenever the pair is within reach, and by no less
otherwise; two particles of one cell always differ by their minimum image.
"""
import numpy as np


def _min_image(d, L):
    return d - L * np.round(d / L)


def _case(rng, na, L):
    w = L / na
    c_idx = rng.integers(0, na, size=3)
    centre = (c_idx + 0.5) * w
    own = centre + rng.uniform(-0.5, 0.5, size=(200, 3)) * w  # inside the cell
    q = rng.uniform(0.0, 1.0, size=(4000, 3)) * L
    reach = w.min() * rng.uniform(0.3, 1.0)  # at most the shortest cell edge
    d = q - centre
    shifted = np.where(d > L / 2, q - L, np.where(d < -L / 2, q + L, q))
    return w, own, q, shifted, reach


def test_shifted_candidate_is_minimum_image_within_reach():
    rng = np.random.default_rng(5)
    for na in (np.array([4, 4, 4]), np.array([4, 6, 10]), np.array([12, 4, 8])):
        L = rng.uniform(0.5, 2.0, size=3)
        for _ in range(20):
            w, own, q, shifted, reach = _case(rng, na, L)
            direct = own[:, None, :] - shifted[None, :, :]
            mini = _min_image(own[:, None, :] - q[None, :, :], L)
            dd = np.sqrt((direct ** 2).sum(-1))
            dm = np.sqrt((mini ** 2).sum(-1))
            near = dm <= reach
            assert near.any()
            assert np.allclose(direct[near], mini[near], rtol=0, atol=1e-12 * L.max())
            assert np.all(dd >= dm - 1e-12 * L.max())
            assert not np.any((dd <= reach) & ~near)


def test_cell_mates_differ_by_their_minimum_image():
    rng = np.random.default_rng(6)
    for na in (np.array([4, 4, 4]), np.array([6, 4, 12])):
        L = rng.uniform(0.5, 2.0, size=3)
        w, own, _, _, _ = _case(rng, na, L)
        d = own[:, None, :] - own[None, :, :]
        assert np.allclose(d, _min_image(d, L), rtol=0, atol=1e-12 * L.max())


def test_the_shift_fails_on_a_one_cell_axis():
    """An axis of one cell (grids take one cell or an even count of at least
    four) breaks the argument: some pair within reach is then found only
    through another image, so such grids keep the per-pair wrap."""
    rng = np.random.default_rng(7)
    na, L = np.array([1, 4, 4]), np.ones(3)
    w, own, q, shifted, _ = _case(rng, na, L)
    reach = 0.2
    direct = own[:, None, :] - shifted[None, :, :]
    mini = _min_image(own[:, None, :] - q[None, :, :], L)
    near = np.sqrt((mini ** 2).sum(-1)) <= reach
    assert np.any(np.abs(direct[near] - mini[near]).max(-1) > 1e-9)
