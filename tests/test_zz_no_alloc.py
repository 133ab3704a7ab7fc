"""fem_step_no_alloc (the entry point for callers that cannot allocate: partial
residuals in the library's static device scratch, eager launches, no graph)
against fem_step through the C ABI: bitwise the same state on two calls in a row,
the second on a smaller mesh (the scratch keeps the first call's contents, which
the second must not see), in FP32 (bit for bit) and FP64 (to rounding: its LDS
sums are floating-point atomics), and across a change of dt."""
import numpy as np
import pytest

from castgen import configs

pytestmark = pytest.mark.gpu


def _cf():
    from paper_1005_3158_amd import castfem as cf
    return cf


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_no_alloc_steps_equal_fem_step_on_two_meshes(prec):
    cf = _cf()
    precision = cf.FEM_PREC_FP32_KAHAN if prec == "fp32" else cf.FEM_PREC_FP64
    for n, steps in ((16, 53), (10, 37)):          # the second call on a smaller mesh
        p = configs.config2(n=n)
        opts = dict(precision=precision, lds_bytes=cf.lds_for_nodes(256, precision=precision))
        ref = cf.Solver(p, **opts)
        new = cf.Solver(p, **opts)
        try:
            dt = 0.9 * ref.stable_dt()
            ref.step(dt, steps)
            cf.fem_step_no_alloc(new.ctx, dt, steps)
            T_ref, H_ref, T_new, H_new = ref.T(), ref.H(), new.T(), new.H()
            e_ref, e_new = ref.energy(), new.energy()
            print("%s %d^3, %d steps: max|T_no_alloc - T_step| = %.3e K, energy residual %.2e (%.2e)"
                  % (prec, n, steps, float(np.max(np.abs(T_new - T_ref))), e_new["residual"], e_ref["residual"]),
                  flush=True)
            if prec == "fp32":
                # fixed-point scatter: order-independent sums, the same bits
                assert np.array_equal(T_new, T_ref) and np.array_equal(H_new, H_ref)
            else:
                # FP64 LDS atomics add in hardware order: equal to rounding (the FP64 path's bar is 1e-8 K)
                assert float(np.max(np.abs(T_new - T_ref))) <= 1e-9
            assert e_new["steps"] == e_ref["steps"] == steps
        finally:
            ref.close()
            new.close()


def test_no_alloc_follows_a_new_dt_and_mixes_with_fem_step():
    cf = _cf()
    p = configs.config2(n=12)
    opts = dict(precision=cf.FEM_PREC_FP32_KAHAN, lds_bytes=cf.lds_for_nodes(512))
    ref = cf.Solver(p, **opts)
    new = cf.Solver(p, **opts)
    try:
        dt = 0.9 * ref.stable_dt()
        for k, (h, n) in enumerate(((dt, 21), (0.5 * dt, 17), (dt, 40))):
            ref.step(h, n)
            if k == 1:
                new.step(h, n)                       # mixed: a graph call in between
            else:
                cf.fem_step_no_alloc(new.ctx, h, n)
        assert np.array_equal(new.T(), ref.T()) and np.array_equal(new.H(), ref.H())
    finally:
        ref.close()
        new.close()


def test_no_alloc_refuses_what_it_does_not_cover():
    cf = _cf()
    p = configs.config2(n=8)
    s = cf.Solver(p, precision=cf.FEM_PREC_FP32_KAHAN, scatter=cf.FEM_SCATTER_COLORED)
    try:
        with pytest.raises(cf.FemError) as e:
            cf.fem_step_no_alloc(s.ctx, 0.5 * s.stable_dt(), 3)
        assert e.value.code == -7          # FEM_E_UNSUPPORTED
        with pytest.raises(cf.FemError) as e:
            cf.fem_step_no_alloc(s.ctx, 10.0 * s.stable_dt(), 3)
        assert e.value.code == -4          # FEM_E_UNSTABLE
    finally:
        s.close()
