"""Host logic of the relaxation-set study driver (no GPU): closed-form
references and the per-geometry summary."""
import math

import study


def test_pipe_reference_is_poiseuille_flux_over_section():
    # mean velocity of Poiseuille flow in a bore, g R^2 / (8 nu), times the bore
    # area pi R^2 over the section A, times nu / g (Darcy) = pi R^4 / (8 A)
    R, A = 13.0, 64
    ubar = R * R / 8.0
    assert math.isclose(study.pipe_reference(R, A), ubar * math.pi * R * R / (A * A), rel_tol=1e-15)


def test_triangle_reference_matches_the_equilateral_flux():
    # equilateral triangle of side l: flux Q = sqrt(3) l^4 g / (320 nu)
    l, A = 200.0, 256
    q = math.sqrt(3.0) * l ** 4 / 320.0
    assert math.isclose(study.triangle_reference(l, A), q / (A * A), rel_tol=1e-15)


def test_channel_force_sets_the_peak_velocity():
    tau, R = 0.8, 20.0
    g = study.channel_force(tau, R)
    nu = (tau - 0.5) / 3.0
    assert math.isclose(g * R * R / (4.0 * nu), study.U_TARGET, rel_tol=1e-12)


def test_set_variants_cover_the_paper_sets():
    labels = [v[0] for v in study.set_variants("")]
    assert labels[:5] == ["SRT", "A", "B", "C", "D"]
    assert sum(1 for v in study.set_variants("") if v[1] == "E") == len(study.SET_E_LAMBDAS)
    assert [v[0] for v in study.set_variants("B,D")] == ["B", "D"]


def test_summary_spread_and_normalisation():
    recs = [dict(geometry="g", label="B", set="B", tau=t, k=k, k_ref=None, iterations_paper=None,
                 iterations_mean2=100) for t, k in ((0.6, 2.0), (1.0, 2.02), (1.6, 2.04))]
    study.normalise(recs)
    assert math.isclose(recs[1]["k_over_ref"], 1.0)
    line = study.summarize(recs).splitlines()[-1]
    assert "1.980%" in line and "None/100" in line
