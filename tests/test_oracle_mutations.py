"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle's source, plants one plausible mistake (a wrong
threshold, a dropped term, a wrong sign, a wrong penalty, a frozen subspace,
a wrong Procrustes factor), loads the copy as a separate module on the CPU,
and checks that the pin battery rejects it, while the unmodified oracle
passes the same battery.
"""

import os
import sys
import types

import numpy as np
import pytest

import workloads
from oracle import default_lambdas, fold, horpca_admm, svt, unfold

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "pasd_oracle.py")


def _load(mutation=None):
    text = open(SRC).read()
    if mutation is not None:
        old, new = mutation
        assert text.count(old) == 1, old
        text = text.replace(old, new)
    name = "pasd_oracle_mutant"
    mod = types.ModuleType(name)
    sys.modules[name] = mod  # dataclasses resolve annotations through sys.modules
    try:
        exec(compile(text, name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def _battery(m):
    rng = np.random.default_rng(0)
    # (a) Procrustes: the polar factor beats random Stiefel points.
    G = rng.standard_normal((4, 6))
    V = rng.standard_normal((2, 6))
    Us = m.polar(G @ V.T)
    best = np.linalg.norm(Us @ V - G)
    for _ in range(500):
        q, _ = np.linalg.qr(rng.standard_normal((4, 2)))
        assert np.linalg.norm(q @ V - G) >= best - 1e-12
    # (b) exact per-iteration optimality conditions (S1), (S3).
    wl = workloads.tucker_workload("mut", (6, 7, 8), (2, 3, 2), 0.1, 7, value_range=(-5, 5),
                                   scale="rms")
    st = m.pasd_init(wl.T, wl.ranks, mu0=0.05)
    for _ in range(25):
        m.pasd_iterate(st, 1)
        mu = st.last["mu"]
        Ysum = sum(st.Y)
        on = st.E != 0
        atol = 1e-9 * mu * 30 + 1e-12
        assert np.all(np.abs(Ysum[on] - np.sign(st.E[on])) <= atol)
        assert np.all(np.abs(Ysum[~on]) <= 1 + atol)
        for n in range(3):
            Yhat = st.last["Y_prev"][n] + mu * (st.T - st.Z[n] - st.last["E_prev"])
            assert np.linalg.norm(st.U[n].T @ unfold(Yhat, n), 2) <= st.lam[n] * (1 + 1e-9)
    # (c) R_n = I_n against the independent full-SVD ADMM.
    T = rng.standard_normal((4, 5, 3))
    T[rng.random(T.shape) < 0.15] += 8
    lam = default_lambdas(T.shape)
    ref = horpca_admm(T, lam, 15, mu0=0.01)
    st = m.pasd_init(T, list(T.shape), lam=lam, mu0=0.01)
    for k in range(15):
        m.pasd_iterate(st, 1)
        np.testing.assert_allclose(st.E, ref[k][1], atol=1e-10)
        for n in range(3):
            np.testing.assert_allclose(st.Z[n], ref[k][0][n], atol=1e-10)
    # (d) recovery of a planted low-rank + sparse tensor (Section 5.1).
    wl = workloads.tucker_workload("mutrec", (30, 30, 30), (3, 3, 3), 0.05, 9,
                                   value_range=(-5, 5), scale="rms")
    st = m.pasd_init(wl.T, wl.ranks)
    while st.k < 600:
        m.pasd_iterate(st, 1)
        if max(st.residual) < 1e-8:
            break
    X, _ = m.pasd_output(st)
    assert np.linalg.norm(X - wl.L) / np.linalg.norm(wl.L) < 1e-6


def test_unmodified_oracle_passes_battery():
    _battery(_load())


MUTATIONS = {
    "shrink_threshold_1_over_mu": ("E_new = prox_l1(H_mean, 1.0 / (mu * N))",
                                   "E_new = prox_l1(H_mean, 1.0 / mu)"),
    "multiplier_uses_next_mu": ("st.Y[n] + mu * (T - Z[n] - E_new)",
                                "st.Y[n] + st.rho * mu * (T - Z[n] - E_new)"),
    "multiplier_sign": ("st.Y[n] + mu * (T - Z[n] - E_new)", "st.Y[n] + mu * (T - Z[n] + E_new)"),
    "svt_threshold_times_mu": ("Vn, s = svt(P, st.lam[n] / mu)", "Vn, s = svt(P, st.lam[n] * mu)"),
    "g_drops_multiplier": ("unfold(T - st.E + st.Y[n] / mu, n)", "unfold(T - st.E, n)"),
    "mean_without_division": ("for n in range(N)) / N", "for n in range(N))"),
    "penalty_growth_squared": ("st.mu = min(st.rho * mu, st.mu_max)",
                               "st.mu = min(st.rho * st.rho * mu, st.mu_max)"),
    "frozen_subspace": ("U_new.append(polar(G[n] @ st.P[n].T))", "U_new.append(st.U[n].copy())"),
    "polar_left_factor_only": ("    return U @ Vt\n", "    return U\n"),
    "estep_uses_old_multiplier_sign": ("T - Z[n] + st.Y[n] / mu for n", "T - Z[n] - st.Y[n] / mu for n"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    mod = _load(MUTATIONS[name])
    with pytest.raises(AssertionError):
        _battery(mod)
