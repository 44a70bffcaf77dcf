"""How far the population-controlled hydrogen-chain trajectory carries a
rounding-sized difference, from two stored runs of the FP64 oracle alone:
the 64-walker, 1000-step run with combs every 20 steps, and the same run
started with one orbital entry of every walker changed by one unit in the
last place (tests/golden/make_hchain_perturbed.py).  The GPU parity test of
that run pins E_mix to 1e-8 Ha over its first 150 steps; this shows that no
implementation that rounds differently from the oracle can be held to that
bound much longer: the oracle itself, one ulp apart, stays within 1e-8 Ha
for 150 steps and parts by more than 1e-6 Ha before the end of the run (a
walker near a node amplifies the difference, then the combs pick other
parents)."""
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _emix(name):
    num, den = [], []
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            p = line.split()
            if p and p[0] == "step":
                num.append(float(p[2]))
                den.append(float(p[3]))
    return np.array(num) / np.array(den)


def test_one_ulp_perturbation_parts_the_oracle_trajectory():
    a = _emix("hchain-M50_W64_T1000.txt")
    b = _emix("hchain-M50_W64_T1000_ulp.txt")
    assert a.size == b.size == 1000 and np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    d = np.abs(a - b)
    assert d[:150].max() <= 1e-8
    part = np.nonzero(d > 1e-6)[0]
    assert part.size and 150 < part[0] < 1000
    print(f"one-ulp start: |dE_mix| <= {d[:150].max():.1e} Ha over 150 steps, "
          f"> 1e-8 from step {int(np.nonzero(d > 1e-8)[0][0])}, > 1e-6 from step {int(part[0])}")
