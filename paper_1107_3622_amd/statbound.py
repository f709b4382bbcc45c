"""Statistical bound of the sort's run time (arXiv 1107.3622, Section 3).

The paper models the mean sorting time over a grid of sizes as

    y = b0 + b1 * n log2(n) + b2 * n

fitted by ordinary least squares. It reports, in the layout of a statistics
package, the coefficients with their standard errors, t and p values and
variance inflation factors, the residual standard deviation, R^2 (plain,
adjusted, predicted from PRESS), the analysis of variance with sequential
sums of squares, and per observation the fit, its standard error and the
(standardized) residual.  Section 3.1 gives the fit for K-sort (eq. 1),
Section 3.2 for Heap sort (eq. 2).  This module computes the same
quantities for any (n, time) grid, so the model can be fitted to timings of
the GPU sort.  It is host-side analysis (numpy and scipy); nothing here
touches the device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Fit:
    n: np.ndarray
    y: np.ndarray
    coef: np.ndarray        # b0, b1 (n log2 n), b2 (n)
    se: np.ndarray
    t: np.ndarray
    p: np.ndarray
    vif: float              # of each of the two regressors (equal for two)
    s: float                # residual standard deviation
    r2: float
    r2_adj: float
    press: float
    r2_pred: float
    ss_reg: float
    ss_res: float
    ss_tot: float
    df_reg: int
    df_res: int
    f: float
    p_f: float
    seq_ss: tuple           # SS of n log2 n alone, then of n given n log2 n
    fit: np.ndarray
    se_fit: np.ndarray
    resid: np.ndarray
    st_resid: np.ndarray
    large: list = field(default_factory=list)  # observations with |standardized residual| > 2

    def predict(self, n) -> np.ndarray:
        n = np.asarray(n, dtype=np.float64)
        return self.coef[0] + self.coef[1] * n * np.log2(n) + self.coef[2] * n


def design(n) -> np.ndarray:
    n = np.asarray(n, dtype=np.float64)
    return np.column_stack([np.ones_like(n), n * np.log2(n), n])


def ols(n, y) -> Fit:
    """OLS fit of y on n log2(n) and n with an intercept."""
    from scipy import stats

    n = np.asarray(n, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    X = design(n)
    N, k = X.shape
    if N <= k:
        raise ValueError("need more observations than coefficients")
    # solve through the QR factors: the regressors are nearly collinear
    # (their correlation is 0.9998), so the normal equations lose digits
    Q, R = np.linalg.qr(X)
    coef = np.linalg.solve(R, Q.T @ y)
    fit = X @ coef
    resid = y - fit
    df_res = N - k
    df_reg = k - 1
    ss_res = float(resid @ resid)
    mse = ss_res / df_res
    s = math.sqrt(mse)
    Rinv = np.linalg.inv(R)
    xtx_inv = Rinv @ Rinv.T
    se = np.sqrt(np.diag(xtx_inv) * mse)
    t = coef / se
    p = 2.0 * stats.t.sf(np.abs(t), df_res)
    ss_tot = float(((y - y.mean()) ** 2).sum())
    ss_reg = ss_tot - ss_res
    r2 = ss_reg / ss_tot
    r2_adj = 1.0 - (ss_res / df_res) / (ss_tot / (N - 1))
    h = np.einsum("ij,jk,ik->i", X, xtx_inv, X)  # leverages
    press = float(((resid / (1.0 - h)) ** 2).sum())
    r2_pred = 1.0 - press / ss_tot
    f = (ss_reg / df_reg) / mse
    p_f = float(stats.f.sf(f, df_reg, df_res))
    # sequential SS: n log2 n alone, then n on top of it
    X1 = X[:, :2]
    c1, *_ = np.linalg.lstsq(X1, y, rcond=None)
    r1 = y - X1 @ c1
    ss1 = ss_tot - float(r1 @ r1)
    seq_ss = (ss1, ss_reg - ss1)
    # VIF of either regressor: 1 / (1 - r^2) with r their correlation
    r = np.corrcoef(X[:, 1], X[:, 2])[0, 1]
    vif = 1.0 / (1.0 - r * r)
    se_fit = np.sqrt(mse * h)
    st_resid = resid / (s * np.sqrt(1.0 - h))
    large = [i + 1 for i in range(N) if abs(st_resid[i]) > 2.0]
    return Fit(n, y, coef, se, t, p, float(vif), s, r2, r2_adj, press, r2_pred, ss_reg, ss_res, ss_tot,
               df_reg, df_res, float(f), p_f, seq_ss, fit, se_fit, resid, st_resid, large)


def report(fr: Fit, name: str = "y") -> str:
    """A text report with the quantities the paper prints for its fits."""
    L = []
    L.append(f"{name} = {fr.coef[0]:.6g} + {fr.coef[1]:.6g} n log2(n) + {fr.coef[2]:.6g} n")
    L.append("")
    L.append(f"{'Predictor':<12}{'Coef':>14}{'SE Coef':>14}{'T':>9}{'P':>8}{'VIF':>10}")
    names = ["Constant", "n log2(n)", "n"]
    for j in range(3):
        vif = "" if j == 0 else f"{fr.vif:10.3f}"
        L.append(f"{names[j]:<12}{fr.coef[j]:14.6g}{fr.se[j]:14.6g}{fr.t[j]:9.2f}{fr.p[j]:8.3f}{vif}")
    L.append("")
    L.append(f"S = {fr.s:.6g}   R-Sq = {100 * fr.r2:.1f}%   R-Sq(adj) = {100 * fr.r2_adj:.1f}%")
    L.append(f"PRESS = {fr.press:.6g}   R-Sq(pred) = {100 * fr.r2_pred:.2f}%")
    L.append("")
    L.append(f"{'Source':<16}{'DF':>4}{'SS':>14}{'MS':>14}{'F':>10}{'P':>8}")
    L.append(f"{'Regression':<16}{fr.df_reg:>4}{fr.ss_reg:14.6g}{fr.ss_reg / fr.df_reg:14.6g}{fr.f:10.2f}{fr.p_f:8.3f}")
    L.append(f"{'Residual Error':<16}{fr.df_res:>4}{fr.ss_res:14.6g}{fr.ss_res / fr.df_res:14.6g}")
    L.append(f"{'Total':<16}{fr.df_reg + fr.df_res:>4}{fr.ss_tot:14.6g}")
    L.append(f"Seq SS: n log2(n) {fr.seq_ss[0]:.6g}, n {fr.seq_ss[1]:.6g}")
    L.append("")
    L.append(f"{'Obs':>4}{'n':>12}{'y':>12}{'Fit':>12}{'SE Fit':>12}{'Residual':>12}{'St Resid':>10}")
    for i in range(len(fr.n)):
        flag = " R" if (i + 1) in fr.large else ""
        L.append(f"{i + 1:>4}{int(fr.n[i]):>12}{fr.y[i]:12.6g}{fr.fit[i]:12.6g}{fr.se_fit[i]:12.6g}"
                 f"{fr.resid[i]:12.6g}{fr.st_resid[i]:10.2f}{flag}")
    return "\n".join(L)
