"""The oracle's multi-threaded run (the CPU timing over all host cores and the
long full-size reference runs) against the serial oracle: the same element
routines with each node's element sum in the serial order, so the two runs must
agree bit for bit, on tets and hexahedra, with fixed temperatures, Robin faces,
matched interfaces and non-matching contact, and for any thread count."""
import numpy as np
import pytest

from castgen import configs


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_tets_with_interfaces_bitwise(orc, threads):
    p = configs.config2(n=9)
    dt = 0.9 * orc.stable_dt(p)
    a = orc.run(p, dt, 40, diag=True)
    b = orc.run_omp(p, dt, 40, diag=True, threads=threads)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_hex_cube_with_fixed_and_robin_faces_bitwise(orc):
    for p in (configs.config1(), configs.config4_trajectory(5003, n=8)):
        dt = 0.9 * orc.stable_dt(p)
        a = orc.run(p, dt, 60, diag=True)
        b = orc.run_omp(p, dt, 60, diag=True, threads=4)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_nonmatching_contact_bitwise(orc):
    p = configs.tet_casting_nonmatching(n_cast=6, n_mold=8, jitter=0.15)
    P = orc.Problem(p)
    dt = 0.9 * orc.stable_dt(P)
    a = orc.run(P, dt, 30, diag=True)
    b = orc.run_omp(P, dt, 30, diag=True, threads=5)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
