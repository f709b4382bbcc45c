"""The statistical-bound fit (y = b0 + b1 n log2 n + b2 n by OLS) pinned to
the paper's own output: run on Table 1 (Section 2), it must reproduce every
figure printed for K-sort in Section 3.1 (eq. 1) and for Heap sort in
Section 3.2 (eq. 2), each to the digits printed."""
import os

import numpy as np

from paper_1107_3622_amd import statbound

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1.txt")


def table1():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([float(x) for x in line.split("|")])
    a = np.array(rows)
    return a[:, 0], a[:, 1], a[:, 2], a[:, 3]


def close(x, printed, decimals):
    """x agrees with a value printed to `decimals` places."""
    return abs(x - printed) <= 0.5 * 10.0 ** (-decimals) + 1e-12


# (coef, se, t, p) per predictor; S, R-Sq, R-Sq(adj), PRESS, R-Sq(pred);
# ANOVA SS and MS, F; sequential SS; per observation fit, SE fit, residual,
# standardized residual.  Values and their printed decimals, Section 3.1.
K_SORT = dict(
    coef=[(0.7516, 4), (0.00000048, 8), (-0.00001048, 8)],
    se=[(0.4153, 4), (0.00000010, 8), (0.00000229, 8)],
    t=[1.81, 4.89, -4.58], p=[0.113, 0.002, 0.003], vif=2225.579,
    s=0.499133, r2=97.0, r2_adj=96.1, press=8.44451, r2_pred=85.42,
    ss=(56.177, 1.744, 57.921), ms=(28.088, 0.249), f=112.74, seq=(50.942, 5.235),
    fit=[0.501, 0.054, -0.163, 0.052, 1.751, 2.709, 3.782, 3.895, 4.356, 7.550],
    se_fit=[0.366, 0.274, 0.238, 0.265, 0.247, 0.217, 0.202, 0.202, 0.209, 0.422],
    resid=[-0.485, 0.027, 0.350, 0.602, 0.163, -0.112, -0.493, -0.445, -0.287, 0.679],
    st=[-1.43, 0.06, 0.80, 1.42, 0.38, -0.25, -1.08, -0.97, -0.63, 2.54], obs_dec=3)

# Section 3.2
HEAP_SORT = dict(
    coef=[(0.12574, 5), (0.00000013, 8), (-0.00000256, 8)],
    se=[(0.06803, 5), (0.00000002, 8), (0.00000037, 8)],
    t=[1.85, 8.29, -6.85], p=[0.107, 0.000, 0.000], vif=2225.579,
    s=0.0817608, r2=99.9, r2_adj=99.8, press=0.225845, r2_pred=99.28,
    ss=(31.169, 0.047, 31.216), ms=(15.585, 0.007), f=2331.34, seq=(30.856, 0.313),
    fit=[0.0907, 0.1055, 0.2186, 0.7985, 2.1379, 2.7507, 3.3958, 3.4618, 3.7289, 5.4832],
    se_fit=[0.0600, 0.0449, 0.0391, 0.0434, 0.0404, 0.0355, 0.0331, 0.0331, 0.0343, 0.0691],
    resid=[-0.0751, 0.0006, 0.0565, 0.0968, 0.0261, -0.0272, -0.0209, -0.0836, -0.0850, 0.1119],
    st=[-1.35, 0.01, 0.79, 1.40, 0.37, -0.37, -0.28, -1.12, -1.14, 2.56], obs_dec=4)


def check(fr, want):
    bad = []
    for j in range(3):
        if not close(fr.coef[j], *want["coef"][j]):
            bad.append(f"coef {j}: {fr.coef[j]}")
        if not close(fr.se[j], *want["se"][j]):
            bad.append(f"se {j}: {fr.se[j]}")
        if not close(fr.t[j], want["t"][j], 2):
            bad.append(f"t {j}: {fr.t[j]}")
        if not close(fr.p[j], want["p"][j], 3):
            bad.append(f"p {j}: {fr.p[j]}")
    for name, got, val, dec in [("vif", fr.vif, want["vif"], 3), ("S", fr.s, want["s"], 7 if want["s"] < 0.1 else 6),
                                ("R-Sq", 100 * fr.r2, want["r2"], 1), ("R-Sq(adj)", 100 * fr.r2_adj, want["r2_adj"], 1),
                                ("PRESS", fr.press, want["press"], 5 if want["press"] > 1 else 6),
                                ("R-Sq(pred)", 100 * fr.r2_pred, want["r2_pred"], 2),
                                ("SS reg", fr.ss_reg, want["ss"][0], 3), ("SS res", fr.ss_res, want["ss"][1], 3),
                                ("SS tot", fr.ss_tot, want["ss"][2], 3),
                                ("MS reg", fr.ss_reg / fr.df_reg, want["ms"][0], 3),
                                ("MS res", fr.ss_res / fr.df_res, want["ms"][1], 3),
                                ("F", fr.f, want["f"], 2), ("Seq SS 1", fr.seq_ss[0], want["seq"][0], 3),
                                ("Seq SS 2", fr.seq_ss[1], want["seq"][1], 3)]:
        if not close(got, val, dec):
            bad.append(f"{name}: {got} vs printed {val}")
    if fr.p_f >= 0.0005:
        bad.append(f"P of F: {fr.p_f}")
    d = want["obs_dec"]
    for i in range(10):
        for name, got, val, dd in [("fit", fr.fit[i], want["fit"][i], d), ("se fit", fr.se_fit[i], want["se_fit"][i], d),
                                   ("resid", fr.resid[i], want["resid"][i], d), ("st resid", fr.st_resid[i], want["st"][i], 2)]:
            if not close(got, val, dd):
                bad.append(f"obs {i + 1} {name}: {got} vs printed {val}")
    if fr.large != [10]:
        bad.append(f"large residuals at {fr.large}, printed: observation 10 only")
    return bad


def test_table1_n_log_n_column():
    n, nlogn, _, _ = table1()
    assert np.allclose(n * np.log2(n), nlogn, rtol=1e-8)


def test_eq1_k_sort():
    n, _, k, _ = table1()
    assert check(statbound.ols(n, k), K_SORT) == []


def test_eq2_heap_sort():
    n, _, _, h = table1()
    assert check(statbound.ols(n, h), HEAP_SORT) == []


def test_eq3_difference():
    # Section 4 subtracts eq. (2) from eq. (1).  Its coefficients of n log2 n
    # (0.00000035) and n (-0.00000792) follow; its printed constant 0.52586 is
    # an arithmetic slip for 0.7516 - 0.12574 = 0.62586.
    n, _, k, h = table1()
    fk, fh = statbound.ols(n, k), statbound.ols(n, h)
    d = fk.coef - fh.coef
    assert close(d[1], 0.00000035, 8) and close(d[2], -0.00000792, 8)
    assert close(round(fk.coef[0], 4) - round(fh.coef[0], 5), 0.62586, 5)
    # the model is linear: the difference fit equals the fit of the differences
    assert np.allclose(statbound.ols(n, k - h).coef, d, rtol=1e-9, atol=1e-15)


def test_planted_mistakes_are_caught():
    # a dropped term or swapped regressor must not reproduce the printed fit
    n, _, k, _ = table1()
    fr = statbound.ols(n, k)
    wrong = statbound.ols(n, k[::-1])
    assert check(wrong, K_SORT) != []
    fr.coef = fr.coef * np.array([1.0, 1.0, 0.9])
    assert check(fr, K_SORT) != []
