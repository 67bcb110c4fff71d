"""Host logic of the nonlinear solver (Sec. 6.1): the residual-based
pseudo-time step control and the forcing term of the inexact Newton steps."""
import pytest

from paper_2507_22195_amd.dirk import PseudoTime, forcing_term


def test_pseudo_time_follows_the_residual_and_is_capped():
    pt = PseudoTime(tau_init=1.0, tau_max=1e8)
    taus = [pt.update(r) for r in (1.0, 0.5, 0.1, 1e-3, 1e-9)]
    # tau_{m+1} = tau_m |R_{m-1}| / |R_m|, first residual sets no step
    assert taus == [1.0, 2.0, 10.0, 1000.0, 1e8]
    assert pt.history == [1.0, 2.0, 10.0, 1000.0, 1e8]
    # a growing residual shrinks the step again
    assert PseudoTime(1.0, 1e8).update(1.0) == 1.0
    q = PseudoTime(4.0, 1e8)
    q.update(1.0)
    assert q.update(2.0) == 2.0
    q.reset()
    assert q.tau == 4.0 and q.history == [4.0]
    with pytest.raises(ValueError):
        PseudoTime(0.0, 1.0)
    with pytest.raises(ValueError):
        PseudoTime(2.0, 1.0)


def test_forcing_term():
    # first step: eta_max; then gamma (|R| / |R_prev|)^2 capped by eta_max
    assert forcing_term(1.0, None, 1e-12) == 0.1
    assert forcing_term(0.1, 1.0, 1e-12) == pytest.approx(0.9 * 0.01)
    assert forcing_term(0.9, 1.0, 1e-12) == 0.1
    # never tighter than what the stopping test can see: tol / (2 |R|)
    assert forcing_term(1e-10, 1.0, 1e-11) == pytest.approx(0.05)
