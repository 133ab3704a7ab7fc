"""Kernel instantiations that read their material tables from global memory:
problems with more than eight materials (here five casting scenarios merged into
one problem, ten materials), in the apparent-capacity form and with
temperature- and time-dependent properties, against the oracle; and the FP32
hexahedron kernel with variable properties.

Tolerances as elsewhere: FP64 1e-8 K, FP32 1e-3 K away from the freezing range
and 0.05 K within 5 K of it.
"""
import numpy as np
import pytest

from castgen import configs

pytestmark = pytest.mark.gpu


def _cf():
    from paper_1005_3158_amd import castfem as cf
    return cf


def _merged_batch():
    """Five disjoint casting scenarios as one problem with ten materials."""
    b = dict(configs.batch(n_scen=5, n_range=(5, 8)))
    b.pop("mat_scenario")
    return b


def _band(T, T_ref, mat=configs.ALLOY):
    band = (T_ref >= mat[3] - 5.0) & (T_ref <= mat[4] + 5.0)
    err = np.abs(T - T_ref)
    return (float(np.max(err[~band])) if np.any(~band) else 0.0,
            float(np.max(err[band])) if np.any(band) else 0.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apparent_form_with_ten_materials(orc, precision):
    cf = _cf()
    p = _merged_batch()
    assert len(p["materials"]) > 8
    dt = 0.9 * orc.stable_dt(p)
    steps = 300
    _, T_ref, _ = orc.run_apparent(p, dt, steps)
    prec = cf.FEM_PREC_FP64 if precision == "fp64" else cf.FEM_PREC_FP32_KAHAN
    s = cf.Solver(p, precision=prec, latent_model=cf.FEM_LATENT_APPARENT)
    try:
        s.step(dt, steps)
        T = s.T()
    finally:
        s.close()
    off, on = _band(T, T_ref)
    print("apparent, ten materials, %s: max|dT| off-front %.3e K, band %.3e K" % (precision, off, on), flush=True)
    if precision == "fp64":
        assert max(off, on) <= 1e-8
    else:
        assert off <= 1e-3 and on <= 0.05


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_variable_properties_with_ten_materials(orc, precision):
    cf = _cf()
    p = _merged_batch()
    vp = dict(k_of_T=[[(550.0, 180.0), (700.0, 95.0)] if q % 2 == 0 else [(0.0, 0.4), (700.0, 1.2)]
                      for q in range(len(p["materials"]))],
              h_of_T=[(100.0, 3.0), (650.0, 0.5)], h_of_t=[(0.0, 1.0), (0.5, 0.3)])
    p["varprops"] = vp
    props = orc.VarProps(len(p["materials"]), **vp)
    dt = 0.9 * orc.stable_dt_var(p, props)
    steps = 300
    _, T_ref, _ = orc.run_var(p, props, dt, steps)
    prec = cf.FEM_PREC_FP64 if precision == "fp64" else cf.FEM_PREC_FP32_KAHAN
    s = cf.Solver(p, precision=prec)
    try:
        s.step(dt, steps)
        T = s.T()
    finally:
        s.close()
    off, on = _band(T, T_ref)
    print("variable properties, ten materials, %s: max|dT| off-front %.3e K, band %.3e K" % (precision, off, on),
          flush=True)
    if precision == "fp64":
        assert max(off, on) <= 1e-8
    else:
        assert off <= 1e-3 and on <= 0.05


def test_variable_properties_fp32_hexahedra(orc):
    cf = _cf()
    p = dict(configs.config1(), varprops=dict(k_of_T=[[(550.0, 180.0), (620.0, 150.0), (700.0, 95.0)]],
                                              dir_of_t=[(0.0, 0.0), (15.0, 250.0), (40.0, 120.0)]))
    props = orc.VarProps(1, **p["varprops"])
    dt = 0.9 * orc.stable_dt_var(p, props)
    _, T_ref, _ = orc.run_var(p, props, dt, 300)
    s = cf.Solver(p, precision=cf.FEM_PREC_FP32_KAHAN, block_elems=512)
    try:
        s.step(dt, 300)
        T = s.T()
    finally:
        s.close()
    off, on = _band(T, T_ref)
    print("variable properties, hex fp32: max|dT| off-front %.3e K, band %.3e K" % (off, on), flush=True)
    assert off <= 1e-3 and on <= 0.05
