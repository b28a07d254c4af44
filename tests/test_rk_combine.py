"""CPU tests of the library's RK accumulation (the compensated combination
U_out = a U_base + b (U_stage + dt L) of the update kernels, csrc/compensated.h).

The header is compiled for the host with hipcc into a small harness
(tests/rk_combine_host.cpp) and checked against exact rational arithmetic: the
compensated form must give the correctly rounded value of the exact combination of
its double inputs, where one rounding per operation (the plain expression) does not.
"""
import math
import os
import shutil
import subprocess
from fractions import Fraction as Fr

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_12240_amd", "csrc")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("rk") / "rk_combine_host")
    subprocess.run([cc, "-x", "hip", "--offload-host-only", "-O2", "-ffp-contract=on", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "rk_combine_host.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, samples):
    out = subprocess.run([exe], input=np.ascontiguousarray(samples, dtype=np.float64).tobytes(),
                         capture_output=True, check=True).stdout
    return np.frombuffer(out, dtype=np.float64).reshape(-1, 2)


def _samples(seed, n):
    rng = np.random.default_rng(seed)
    a = rng.choice([0.0, 0.5, 1.0, 0.3], n)
    b = np.where(a == 0.0, 1.0, np.where(a == 0.5, 0.5, rng.uniform(0.1, 1.0, n)))
    ub = rng.uniform(0.5, 2.0, n) * 10.0 ** rng.integers(-3, 4, n) * rng.choice([-1.0, 1.0], n)
    us = ub * (1.0 + rng.normal(0.0, 1e-3, n))
    dt = rng.uniform(1e-4, 1e-2, n)
    L = us * rng.normal(0.0, 1.0, n) * 10.0 ** rng.integers(-9, 1, n)
    return np.stack([a, ub, b, us, dt, L], axis=1)


def test_compensated_combination_is_correctly_rounded(harness):
    x = _samples(12240, 6000)
    r = _run(harness, x)
    exact_c = plain_c = 0
    worst = Fr(0)
    for (a, ub, b, us, dt, L), (comp, plain) in zip(x, r):
        ex = Fr(a) * Fr(ub) + Fr(b) * (Fr(us) + Fr(dt) * Fr(L))
        cr = float(ex)                                   # the correctly rounded value
        exact_c += comp == cr
        plain_c += plain == cr
        worst = max(worst, abs(Fr(comp) - ex) / Fr(math.ulp(cr)))
    assert exact_c == len(x), (exact_c, len(x))
    assert worst <= Fr(1, 2)
    # the plain expression rounds several times (a mistake that dropped the error
    # terms would make the compensated form look like this)
    assert plain_c < 0.95 * len(x), plain_c


def test_uniform_state_is_exact(harness):
    # L = 0 and U_base = U_stage: both stages of SSP-RK2 return the state bit for bit
    v = np.array([1.0, -3.25e-7, 7.5e12, 1e-300, 0.1])
    x = np.stack([np.full_like(v, 0.5), v, np.full_like(v, 0.5), v, np.full_like(v, 1e-3), np.zeros_like(v)], 1)
    x = np.concatenate([x, np.stack([np.zeros_like(v), v, np.ones_like(v), v, np.full_like(v, 1e-3),
                                     np.zeros_like(v)], 1)])
    r = _run(harness, x)
    assert (r[:, 0] == np.concatenate([v, v])).all()


def test_zero_weight_base_is_not_read(harness):
    # a == 0: the base term is absent, so a non-finite U_base does not leak in
    x = np.array([[0.0, np.nan, 1.0, 2.0, 1e-2, 3.0], [0.0, np.inf, 1.0, -1.0, 1e-3, 0.5]])
    r = _run(harness, x)
    assert r[0, 0] == float(Fr(2.0) + Fr(1e-2) * Fr(3.0))
    assert r[1, 0] == float(Fr(-1.0) + Fr(1e-3) * Fr(0.5))


def _rk2(exe, u0, dt, rates):
    inp = np.concatenate([[u0, dt], np.asarray(rates, dtype=np.float64).ravel()]).tobytes()
    out = subprocess.run([exe, "rk2"], input=inp, capture_output=True, check=True).stdout
    return np.frombuffer(out, dtype=np.float64)


def test_many_steps_follow_the_once_rounded_recurrence(harness):
    """Over 1500 SSP-RK2 steps the compensated state is exactly the recurrence that
    rounds each stored stage value once (to nearest double) from the exact stage
    combination; the plain expression departs from it. This is what the in-register
    compensation buys: no rounding inside a substep. It carries nothing across
    substeps, so the once-per-substep rounding itself still accumulates (a steady
    rate rounds the same way every step)."""
    rng = np.random.default_rng(2108)
    for _ in range(4):
        n = 1500
        u0, dt = float(rng.uniform(0.5, 2.0)), float(rng.uniform(1e-4, 1e-2))
        rates = rng.normal(0.0, 1.0, (n, 2)) * 10.0 ** float(rng.integers(-9, -3))
        comp, plain = _rk2(harness, u0, dt, rates)
        u, h = Fr(u0), Fr(dt)
        for l1, l2 in rates:
            u1 = Fr(float(u + h * Fr(l1)))
            u = Fr(float(Fr(1, 2) * u + Fr(1, 2) * (u1 + h * Fr(l2))))
        assert comp == float(u)
        assert plain != float(u)
