"""Seeded synthetic inputs (CPU): the same seed gives the same input, shapes and
statistics follow the configurations, and the flat parameter layout splits
and joins without loss."""
import numpy as np

import workloads as W


def test_config0_is_deterministic_and_shaped():
    a = W.config0()
    b = W.config0()
    spec, params, system, opts = a
    assert np.array_equal(params, b[1]) and np.array_equal(system.pos, b[2].pos)
    assert system.n == 512 and spec.n_params == params.size
    assert np.allclose(system.box, 512 ** (1 / 3) / 33.4 ** (1 / 3), rtol=1e-9)
    assert np.all(system.vel == 0.0)
    # weights N(0, 0.1^2) for every parameter (reading of the configs)
    assert abs(params.std() - 0.1) < 0.01 and abs(params.mean()) < 0.01


def test_config1_density_and_temperature():
    spec, params, system, opts = W.config1()
    assert system.n == 216000
    rho = system.n / np.prod(system.box)
    assert abs(rho - W.WATER_DENSITY) < 1e-9 * W.WATER_DENSITY
    kB = 8.617333262e-5
    ke = 0.5 * W.WATER_MASS * (system.vel ** 2).sum() / 9.648533212e-5
    T = 2 * ke / (3 * system.n * kB)
    assert abs(T - 300.0) < 3.0
    assert np.allclose(system.vel.mean(axis=0), 0.0, atol=1e-9)   # no centre-of-mass drift


def test_parameter_layout_round_trip():
    for spec in (W.water_spec(30), W.aacg_gold_spec(50), W.c60_spec(30)):
        p = np.arange(spec.n_params, dtype=np.float64)
        parts = spec.split(p)
        assert np.array_equal(spec.join(parts), p)
        # flat order: w0, b0, w1, b1, c^R, c^A
        assert parts["w0"].ravel()[0] == 0 and parts["cA"].ravel()[-1] == spec.n_params - 1


def test_fitness_and_serving_inputs_are_deterministic():
    f1 = W.config3(n_candidates=3, n_structures=10, size_range=(32, 100))
    f2 = W.config3(n_candidates=3, n_structures=10, size_range=(32, 100))
    for s1, s2 in zip(f1.systems, f2.systems):
        assert np.array_equal(s1.pos, s2.pos) and np.array_equal(s1.types, s2.types)
    assert np.array_equal(f1.candidates[0][0], f1.base_params[0])     # candidate 0 is the base set
    assert np.all(f1.family[:5] == 0) and np.all(f1.family[5:] == 1)
    s1 = W.config4(n_replicas=4, n_requests=50, size_range=(100, 200))
    s2 = W.config4(n_replicas=4, n_requests=50, size_range=(100, 200))
    assert np.array_equal(s1.arrivals_s, s2.arrivals_s) and np.array_equal(s1.replica_of, s2.replica_of)
    assert np.all(np.diff(s1.arrivals_s) > 0)
