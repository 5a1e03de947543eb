"""Write config1_oracle.json: oracle results on the 12-atom solute in 207
waters (18.6 A box, cutoff 9 A, DSF alpha 0.2, 1 A switch), both lambda
schedules at five lambdas.

Only the oracle computes the stored values; the seeded generator provides
the inputs (a fingerprint of them is stored so that a test can tell a
changed generator from a changed oracle).  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2608_12691_amd import systems as S  # noqa: E402

LAMBDAS = (0.0, 0.3, 0.5, 0.75, 1.0)
SCHEDULES = {"beutler": O.BEUTLER, "lbf": O.LBF}
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_oracle.json")


def force_atoms(system):
    """Every solute atom, the first 12 solvent atoms and 12 seeded others."""
    sol = np.nonzero(system.is_solute)[0]
    rest = np.nonzero(system.is_solute == 0)[0]
    rng = np.random.default_rng(12691)
    extra = rng.choice(rest[12:], size=12, replace=False)
    return sorted(int(i) for i in np.concatenate([sol, rest[:12], extra]))


def fingerprint(system):
    p = np.asarray(system.positions, dtype=np.float64)
    return dict(n_atoms=int(p.shape[0]), sum=float(p.sum()), sum_sq=float((p * p).sum()),
                first=[float(v) for v in p[0]], last=[float(v) for v in p[-1]],
                n_solute=int(np.sum(system.is_solute)), n_exclusions=int(np.asarray(system.exclusions).shape[0]),
                box=[float(v) for v in system.box])


def main():
    w = S.make_config(1)
    s = w.systems[0]
    atoms = force_atoms(s)
    cases = []
    for name, sched in SCHEDULES.items():
        P = O.Params.of(w, sched)
        for lam in LAMBDAS:
            r = O.evaluate_system(s, w.ff, P, lam)
            F = r["forces"]
            cases.append(dict(schedule=name, lam=lam, terms=[float(v) for v in r["terms"]],
                              abs_terms=[float(v) for v in r["abs_terms"]], n_pairs=int(r["n_pairs"]),
                              forces=[[float(v) for v in F[a]] for a in atoms],
                              force_sq_sum_all=float(np.sum(F * F))))
    doc = dict(
        _about="Oracle results (oracle/ only) on the seeded 12-atom-solute water box; written by make_golden.py",
        workload=dict(name=w.name, seed=w.seed, cutoff=w.cutoff, switch_width=w.switch_width,
                      dsf_alpha=w.dsf_alpha, sc_alpha=w.sc_alpha),
        inputs=fingerprint(s),
        force_atoms=atoms,
        cases=cases,
    )
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote", OUT, len(cases), "cases,", len(atoms), "force atoms")


if __name__ == "__main__":
    main()
