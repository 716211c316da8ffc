"""The FP64 energy parity rule, shared by the GPU tests and the benchmark's
oracle comparison -- TEST INFRASTRUCTURE ONLY (no method arithmetic: it
compares final energies and directions that the callers computed).

Bar: final kinetic energy within |dK| <= 1e-8 K + 1e-12 MeV for at least
99.9% of the born electrons, and the same forward / backward direction for at
least 99.9%; birth times are compared separately (1e-10 of max(|t|, T)).

The result the oracle defines is the RK4 discretization in exact arithmetic.
The double oracle itself misses it by more than 1e-8 for a few electrons in
ten thousand (trajectories that amplify rounding by up to ~1e8), so the rule
uses two references, and no electron is excluded from either:

  (1) identical inputs: the GPU's energies against the double oracle's push
      of the same electrons from the GPU's own birth times and positions;
  (2) exact answer: the GPU's energies against the oracle built in x87
      extended precision (2^11 finer rounding), running its own chain from
      the seed (or its push from the same inputs, for stage tests);
  (3) the forward / backward flags agree with the double oracle's.

Each must hold for >= 99.9% of the electrons.  The report also gives the
double oracle's own agreement with the extended one (when the caller has the
double oracle's chain), which shows where the bar sits for double arithmetic.
"""
from __future__ import annotations

import numpy as np

REL_TOL = 1e-8
ABS_TOL_MEV = 1e-12
BAR = 0.999


def within(K, Kref):
    """|K - Kref| <= 1e-8 Kref + 1e-12 MeV, elementwise."""
    K, Kref = np.asarray(K, dtype=np.float64), np.asarray(Kref, dtype=np.float64)
    return np.abs(K - Kref) <= REL_TOL * np.abs(Kref) + ABS_TOL_MEV


def allowed_misses(n, bar=BAR):
    """Largest number of misses that still leaves a fraction >= bar of n."""
    return int(np.floor((1.0 - bar) * n + 1e-9))


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def fp64_energy_verdict(Kg, fg, Kop, fop, Kx=None, Koc=None):
    """Kg, fg: GPU energies [MeV] and forward flags; Kop, fop: the double
    oracle's push from the same inputs; Kx: the extended-precision oracle's
    energies (or None); Koc: the double oracle's own chain (or None, report
    only).  All for the same born electrons in the same order.  Returns a dict
    of counts and fractions and `passed` (rules (1)-(3))."""
    Kg, Kop = np.asarray(Kg, dtype=np.float64), np.asarray(Kop, dtype=np.float64)
    n = Kg.size
    ok1 = within(Kg, Kop)
    same = np.asarray(fg) == np.asarray(fop)
    out = dict(electrons=n, allowed_misses=allowed_misses(n),
               frac_vs_oracle=float(ok1.mean()) if n else 1.0,
               misses_vs_oracle=int((~ok1).sum()),
               max_rel_vs_oracle=float(_rel(Kg, Kop).max()) if n else 0.0,
               median_rel_vs_oracle=float(np.median(_rel(Kg, Kop))) if n else 0.0,
               same_direction=float(same.mean()) if n else 1.0,
               direction_misses=int((~same).sum()))
    passed = out["misses_vs_oracle"] <= out["allowed_misses"] and \
        out["direction_misses"] <= out["allowed_misses"]
    if Kx is not None:
        Kx = np.asarray(Kx, dtype=np.float64)
        ok2 = within(Kg, Kx)
        out.update(frac_vs_extended=float(ok2.mean()) if n else 1.0,
                   misses_vs_extended=int((~ok2).sum()),
                   max_rel_vs_extended=float(_rel(Kg, Kx).max()) if n else 0.0)
        passed = passed and out["misses_vs_extended"] <= out["allowed_misses"]
        if Koc is not None:
            oo = within(np.asarray(Koc, dtype=np.float64), Kx)
            out.update(oracle_frac_vs_extended=float(oo.mean()) if n else 1.0,
                       oracle_misses_vs_extended=int((~oo).sum()))
    out["passed"] = bool(passed)
    return out


def summary(v, label=""):
    """One line for a log."""
    s = (f"[parity{label}] {v['electrons']} electrons (<= {v['allowed_misses']} misses allowed): "
         f"same inputs as the double oracle {v['frac_vs_oracle']:.5f} "
         f"({v['misses_vs_oracle']} misses, max rel {v['max_rel_vs_oracle']:.1e})")
    if "frac_vs_extended" in v:
        s += (f"; extended oracle {v['frac_vs_extended']:.5f} ({v['misses_vs_extended']} misses, "
              f"max rel {v['max_rel_vs_extended']:.1e})")
    if "oracle_frac_vs_extended" in v:
        s += (f"; the double oracle's own chain vs extended {v['oracle_frac_vs_extended']:.5f} "
              f"({v['oracle_misses_vs_extended']} misses)")
    s += f"; same direction {v['same_direction']:.5f}"
    return s
