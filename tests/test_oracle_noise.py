"""The force-noise comparison of Sec. III.B.3 on the oracle: the oscillating
cylinder at 1/5 scale (400x160, R=8, period 800 steps), FP64.

Noise is the RMS of a force component minus its centred 41-step moving
average over steps 700..1500 (the short time scale the paper attributes to
the impulsive covered/uncovered terms). The paper states two orderings,
checked here:
* the comoving-frame force (Eq. ForceInMovementMovingFrame) is much less
  noisy than the lattice-frame force (Eq. ForceInMovement): less than half
  its lift-direction noise, for every refill rule;
* the refills of Lallemand & Luo and of Aidun et al. give lower noise than
  the equilibrium at the neighbours' mean.
"""
import numpy as np
import pytest

import lbm_workloads as W
from oracle_helpers import make_oracle, me_series


def force_noise(x, win=41):
    k = np.ones(win) / win
    r = x[win // 2: len(x) - win // 2] - np.convolve(x, k, mode="valid")
    return float(np.sqrt((r * r).mean()))


@pytest.fixture(scope="module")
def noise_by_refill():
    out = {}
    for refill in ("mean", "aidun", "extrapolate"):
        w = W.channel_oscillating_f32(scale=5)
        w["storage"] = "f64"
        w["bodies"][0]["refill"] = refill
        o = make_oracle(w)
        o.step(1500)
        rec = o.records(0)
        sl = slice(700, 1500)
        out[refill] = {mode: [force_noise(me_series(rec, mode)[0][sl, a]) for a in (0, 1)]
                       for mode in ("lattice", "comoving", "lattice_backward")}
    return out


def test_comoving_force_is_less_noisy(noise_by_refill):
    for refill, n in noise_by_refill.items():
        print(refill, {m: [f"{v:.2e}" for v in vals] for m, vals in n.items()})
        assert n["comoving"][1] < 0.5 * n["lattice"][1], refill
        assert n["comoving"][0] <= n["lattice"][0] * 1.0001, refill


def test_extrapolation_and_aidun_refills_are_less_noisy(noise_by_refill):
    base = noise_by_refill["mean"]["comoving"]
    for refill in ("aidun", "extrapolate"):
        n = noise_by_refill[refill]["comoving"]
        assert n[0] < base[0] and n[1] < base[1], (refill, n, base)
