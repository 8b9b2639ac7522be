"""Host logic of the Section 6.2 scaling experiments: the delay moments the
error is fitted against, pinned to the paper's printed mean delays and to
closed forms of the uniform-delay moments, the workload builders, and the
fit helpers on data with a known answer."""
from fractions import Fraction

import pytest

from paper_2404_03399_amd import experiments as X
from paper_2404_03399_amd import workloads as W


def test_mean_delays_printed_in_section_6():
    # Sec. 6.2: probability sets {0.5,0.3,0.2}, {0.3,0.4,0.3}, {0,0,1} give
    # mean delays 0.7, 1.0 and 2.0
    assert X.mean_delay(("0.5", "0.3", "0.2")) == Fraction(7, 10)
    assert X.mean_delay(("0.3", "0.4", "0.3")) == 1
    assert X.mean_delay(("0", "0", "1")) == 2


@pytest.mark.parametrize("L", range(1, 9))
def test_uniform_delay_moments_closed_forms(L):
    probs = W.uniform_probs(L)
    assert sum(Fraction(p) for p in probs) == 1
    # AT2: E[k^2] + E[k] = (L^2 - 1) / 3, the (L^2 - 1) law of Sec. 6.2
    assert X.delay_moment(probs, 2) == Fraction(L * L - 1, 3)
    # AT4: E[k^4] + 6E[k^3] + 11E[k^2] + 6E[k] = E[k(k+1)(k+2)(k+3)]
    #      = (L-1)(L+1)(L+2)(L+3)/5 for p_k = 1/L (hockey-stick identity)
    assert X.delay_moment(probs, 4) == Fraction((L - 1) * (L + 1) * (L + 2) * (L + 3), 5)
    # the moment polynomial itself, term by term
    m = [sum(Fraction(1, L) * k ** i for k in range(L)) for i in range(5)]
    assert X.delay_moment(probs, 4) == m[4] + 6 * m[3] + 11 * m[2] + 6 * m[1]
    assert X.delay_moment(probs, 2) == m[2] + m[1]


def test_fit_helpers_on_exact_data():
    xs = [2, 4, 8, 16, 32]
    assert X.loglog_slope(xs, [3.0 * x ** -2 for x in xs]) == pytest.approx(-2.0, abs=1e-12)
    fit = X.linear_fit([0.0, 1.0, 2.5, 5.0], [1.0 + 0.5 * x for x in (0.0, 1.0, 2.5, 5.0)])
    assert fit["c0"] == pytest.approx(1.0) and fit["c1"] == pytest.approx(0.5) and fit["r2"] == pytest.approx(1.0)


def test_scaling_workloads():
    ws, grp = W.error_vs_pe_workloads("at2", 256, X.PE_COUNTS, 3)
    assert len(ws) == 15 and grp == [g for g in range(5) for _ in range(3)]
    assert len({w.seed for w in ws}) == 15
    assert [w.n_elem // w.pe_size for w in ws[::3]] == list(X.PE_COUNTS)
    w = ws[0]
    assert (w.degree, w.rk, w.scheme, w.per_stage, w.probs) == (1, "heun", "adg_at", False, W.DELAYS_FIG9)
    # sigma = a dt / dx <= 0.1 and T = 1 reached exactly
    assert w.dt * w.n_steps == pytest.approx(1.0, rel=1e-14)
    assert w.dt / (W.TWO_PI / 256) <= 0.1 + 1e-12
    ws, grp = W.error_vs_delay_workloads("at4", 128, 16, (1, 2, 3), 2)
    assert [len(w.probs) for w in ws] == [1, 1, 2, 2, 3, 3] and {w.degree for w in ws} == {3}
    assert len({w.n_steps for w in ws}) == 1
