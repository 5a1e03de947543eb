"""Write closed_forms.json: single-pair values of the alchemical pair
potential evaluated in 40-digit arithmetic (mpmath), independently of the
oracle (this script never imports it).

Energies follow the defining formulas:
- plain pair: 4 eps [(s/r)^12 - (s/r)^6] S(r) + k_e qq D(r);
- Beutler soft core (the conventional form the paper contrasts with LBF,
  Linear Basis Function section): lv 4 eps (x^2 - x) S(r) + le k_e qq D(r),
  x = 1 / (a (1 - lv) + (r/s)^6), lv = min(1, 2 lam), le = max(0, 2 lam - 1);
- LBF (eq. 4 with eqs. 5-10): hA [LJ S + k_e qq D] + hB eps u_cap(r/s) S,
  hA = S32((lam - 0.35)/0.65), hB = S22(lam) - hA;
- S(r) = 1 - S22((r - r_s)/w) on (r_s, r_c) (eq. 9 as the switch), D(r) the
  damped shifted-force kernel.
Derivatives (-du/dr, du/dlam, du/dsig, du/deps, du/dqq) are taken by
mpmath's numerical differentiation of those energies at 40 digits, one-sided
from the left in lambda (the Beutler schedule has a kink at lambda = 1/2,
and the left derivative is the convention), so they test the oracle's
hand-written derivatives against a route that shares nothing with them.

    python tests/golden/make_closed_forms.py    # rewrites closed_forms.json
"""
import json
import os

import mpmath as mp

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "closed_forms.json")
DPS = 40
# constants are set by _constants() at the working precision, whatever
# precision the caller's mpmath context had when this module was imported
KE = RC = W = ALPHA = SCA = SIG = EPS = QQ = None


def _constants():
    global KE, RC, W, ALPHA, SCA, SIG, EPS, QQ
    KE = mp.mpf("332.06371")
    RC, W, ALPHA, SCA = mp.mpf(9), mp.mpf(1), mp.mpf("0.2"), mp.mpf("0.5")
    SIG, EPS, QQ = mp.mpf("3.2"), mp.mpf("0.12"), mp.mpf("-0.3")


def s22(x):
    return 6 * x ** 5 - 15 * x ** 4 + 10 * x ** 3


def s32(x):
    return mp.mpf(0) if x <= 0 else 10 * x ** 6 - 24 * x ** 5 + 15 * x ** 4


def switch(r):
    rs = RC - W
    if r <= rs:
        return mp.mpf(1)
    return 1 - s22((r - rs) / W)


def dsf(r):
    ec = mp.erfc(ALPHA * RC)
    slope = ec / RC ** 2 + 2 * ALPHA / mp.sqrt(mp.pi) * mp.exp(-(ALPHA * RC) ** 2) / RC
    return mp.erfc(ALPHA * r) / r - ec / RC + slope * (r - RC)


def lj(r, s, e):
    return 4 * e * ((s / r) ** 12 - (s / r) ** 6)


def ucap(x):
    if x < 1:
        return -868 * x ** 6 + mp.mpf("2188.8") * x ** 5 - 1440 * x ** 4 + mp.mpf("119.2")
    return 4 * x ** -12 - 4 * x ** -6


def u_plain(r, lam, s, e, qq):
    return lj(r, s, e) * switch(r) + KE * qq * dsf(r)


def u_beutler(r, lam, s, e, qq):
    lv = min(mp.mpf(1), 2 * lam)
    le = max(mp.mpf(0), 2 * lam - 1)
    x = 1 / (SCA * (1 - lv) + (r / s) ** 6)
    return lv * 4 * e * (x * x - x) * switch(r) + le * KE * qq * dsf(r)


def u_lbf(r, lam, s, e, qq):
    hA = s32((lam - mp.mpf("0.35")) / mp.mpf("0.65"))
    hB = s22(lam) - hA
    return hA * (lj(r, s, e) * switch(r) + KE * qq * dsf(r)) + hB * e * ucap(r / s) * switch(r)


FORMS = {"plain": u_plain, "beutler": u_beutler, "lbf": u_lbf}


def row(form, r, lam):
    f = FORMS[form]
    r, lam = mp.mpf(r), mp.mpf(lam)
    u = f(r, lam, SIG, EPS, QQ)
    mdr = -mp.diff(lambda v: f(v, lam, SIG, EPS, QQ), r)
    dl = mp.diff(lambda v: f(r, v, SIG, EPS, QQ), lam, direction=-1)
    ds = mp.diff(lambda v: f(r, lam, v, EPS, QQ), SIG)
    de = mp.diff(lambda v: f(r, lam, SIG, v, QQ), EPS)
    dq = mp.diff(lambda v: f(r, lam, SIG, EPS, v), QQ)
    return [float(v) for v in (u, mdr, dl, ds, de, dq)]


def table():
    with mp.workdps(DPS):
        _constants()
        return _table()


def _table():
    rows = []
    for form in ("beutler", "lbf"):
        for r in ("1.6", "2.0", "2.9", "3.5", "3.6", "8.5", "8.6"):
            for lam in ("0.2", "0.25", "0.4", "0.5", "0.7", "0.75", "0.95", "1.0"):
                rows.append(dict(form=form, r=float(r), lam=float(lam), values=row(form, r, lam)))
    for r in ("2.9", "3.5", "8.5", "8.6"):
        rows.append(dict(form="plain", r=float(r), lam=0.5, values=row("plain", r, "0.5")))
    hl = []
    for lam in ("0.2", "0.35", "0.5", "0.75", "0.9"):
        x = mp.mpf(lam)
        hA = lambda v: s32((v - mp.mpf("0.35")) / mp.mpf("0.65"))
        hB = lambda v: s22(v) - hA(v)
        hl.append(dict(lam=float(lam), values=[float(hA(x)), float(hB(x)), float(mp.diff(hA, x, direction=-1)),
                                                float(mp.diff(hB, x, direction=-1))]))
    return dict(
        _about="Single-pair closed forms in 40-digit arithmetic by tests/golden/make_closed_forms.py (mpmath; "
               "never imports the oracle). values = [u, -du/dr, du/dlambda (left), du/dsigma, du/deps, du/dqq].",
        cite="pair potential: Linear Basis Function section, eqs. 4-10 (LBF) and the conventional soft core it "
             "contrasts (Beutler, exponents 1 and 6, alpha 0.5); switch eq. 9; damped shifted-force Coulomb; "
             "Lorentz-Berthelot combination; left lambda derivative at the Beutler kink",
        params=dict(sigma=float(SIG), epsilon=float(EPS), qq=float(QQ), cutoff=float(RC), switch_width=float(W),
                    dsf_alpha=float(ALPHA), sc_alpha=float(SCA), k_e=float(KE)),
        pairs=rows,
        lbf_switches=dict(cite="eqs. 7-10: [hA, hB, dhA/dlambda, dhB/dlambda]", rows=hl))


if __name__ == "__main__":
    with open(OUT, "w") as fh:
        json.dump(table(), fh, indent=1)
    print("wrote", OUT)
