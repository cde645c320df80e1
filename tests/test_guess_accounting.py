"""Build accounting of the learned-guess SCF (host logic, no GPU).

The run itself never sees the reference energy; afterwards a run that
converged to another state counts as a failure with the plain core-guess
run's builds on top, and a fallback run's builds add to the failed run's.
"""
from paper_2506_06661_amd import guess

E_REF = -11.0
CORE = [(-10.9, 1e-2, False), (-10.9999995, 1e-5, False), (-11.0, 1e-8, True)]  # reaches it at build 2


def test_learned_run_reaches_reference():
    out = {"records": [(-10.99999999, 1e-6, False), (-11.0, 1e-8, True)], "fallback": False,
           "reason": None, "fallback_records": []}
    assert guess.account(out, E_REF, CORE) == {"builds": 1, "wrong_state": False}


def test_other_state_counts_core_run_on_top():
    out = {"records": [(-10.0, 1e-3, False), (-10.5, 1e-4, False), (-10.5, 1e-8, True)], "fallback": False,
           "reason": None, "fallback_records": []}
    acc = guess.account(out, E_REF, CORE)
    assert acc == {"builds": 3 + 2, "wrong_state": True}


def test_fallback_builds_add_up():
    out = {"records": [(-9.0, 1.0, False)] * 4, "fallback": True, "reason": "not converged",
           "fallback_records": CORE}
    assert guess.account(out, E_REF, CORE) == {"builds": 4 + 2, "wrong_state": False}
    out = {"records": [], "fallback": True, "reason": "non-finite guess", "fallback_records": CORE}
    assert guess.account(out, E_REF, CORE)["builds"] == 2
