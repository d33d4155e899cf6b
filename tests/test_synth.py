"""Seeded problem generator: determinism, agent subsets, shapes and ranges."""
import numpy as np
import pytest

from paper_2510_12717_amd import synth


def test_deterministic_and_subset_reproduces():
    a = synth.small_humanoid_batch(6)
    b = synth.small_humanoid_batch(6)
    for k in ("A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu", "stance"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k))
    sub = synth.small_humanoid_batch(agent_ids=[4, 1])
    ref = a.subset([4, 1])
    for k in ("A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu", "stance"):
        np.testing.assert_array_equal(getattr(sub, k), getattr(ref, k))


def test_config_streams_differ():
    a = synth.small_humanoid_batch(2)
    b = synth.humanoid_batch(2)
    assert not np.array_equal(a.A, b.A)


def test_shapes_and_ranges_small_humanoid():
    b = synth.small_humanoid_batch(16)
    s = b.shapes[0]
    assert (s.N, s.nx, s.nu, s.m) == (10, 48, 30, 38)
    A = b.A.reshape(16, 10, 48, 48)
    G = (A - np.eye(48)) / synth.DT
    assert abs(G.std() - 1 / np.sqrt(48)) < 0.01
    Bm = b.B.reshape(16, 10, 48, 30) / synth.DT
    assert abs(Bm.std() - 1 / np.sqrt(30)) < 0.01
    assert abs(b.c.std() - 1e-3) < 1e-4
    lq, lr = np.log10(b.q), np.log10(b.r)
    assert lq.min() >= -2 and lq.max() <= 2 and lr.min() >= -4 and lr.max() <= -1
    assert b.tau_max.min() >= 20 and b.tau_max.max() <= 100
    assert b.mu.min() >= 0.4 and b.mu.max() <= 1.0
    assert abs(b.stance.mean() - 0.6) < 0.06
    assert b.x_ref.size == 16 * 11 * 48


def test_uneven_config_mix():
    shapes = synth.uneven_batch_shapes(400)
    Ns = np.array([s.N for s in shapes])
    assert Ns.min() == 5 and Ns.max() == 20
    kinds = np.array([s.nx for s in shapes])
    assert 0.4 < (kinds == 48).mean() < 0.6
    quad = [s for s in shapes if s.nx == 36][0]
    assert (quad.nu, quad.n_feet, quad.foot_dim, quad.m) == (24, 4, 3, 40)
    b = synth.uneven_batch(12)
    off = b.offsets()
    assert off["A"][-1] == b.A.size and off["stance"][-1] == b.stance.size


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_condition_sweep(kappa):
    b = synth.conditioned_humanoid_batch(8, kappa=kappa)
    q = b.q.reshape(8, 48)
    r = b.r.reshape(8, 30) / 10 ** -2.5
    assert q.max() / q.min() <= kappa * (1 + 1e-12)
    assert r.max() / r.min() <= kappa * (1 + 1e-12)
    assert q.max() / q.min() > kappa ** 0.8


def test_step_noise_is_per_step():
    b = synth.humanoid_batch(3)
    n0, n1 = synth.step_noise(b, 0), synth.step_noise(b, 1)
    assert n0.shape == (3 * 48,) and not np.array_equal(n0, n1)
    np.testing.assert_array_equal(n0, synth.step_noise(b, 0))
