"""Closed-form solutions of the paper's two transport test cases (§5.1, §5.2).

TEST INFRASTRUCTURE.  Both cases have the exact pressure u = 1 - x, so the
matrix velocity is (1, 0) and all the error of the scheme comes from the
upwind transport.

§5.1 (one fracture, transient, equation test_traceur): fracture from (0, 1/4)
with slope tan(theta); beta = sin(theta)/d_f, k = Lambda_f cos^2(theta).

§5.2 (four fractures, stationary, equation test_traceur4frac):
beta_1 = sin(theta_1)/d_f,1, k_1 = Lambda_f,1 cos^2(theta_1),
beta_2 = cos(theta_2)/d_f,3, k_2 = Lambda_f,3 cos(theta_2) sin(theta_2),
r = Lambda_f,3 d_f,3 sin(theta_2) / (Lambda_f,1 d_f,1 cos(theta_1)).

Reading of a printed typo: in c_{f,3}, the exponents carry
-beta_1/(4 k_1 tan(theta_1)) as printed; integrating the fracture ODE
-k_2 c' + beta_2 c = beta_2 c_{m,3} with the source c_{f,1}((y - 1/4)/tan(theta_1))
gives +beta_1/(4 k_1 tan(theta_1)).  This module uses the sign the ODE fixes;
the test-suite checks it against a numerical integration of the same ODE.
"""
from __future__ import annotations

import math

import numpy as np


class E1:
    def __init__(self, tan_theta=0.5, lam_f=20.0, df=0.01):
        th = math.atan(tan_theta)
        self.tan = tan_theta
        self.beta = math.sin(th) / df
        self.k = lam_f * math.cos(th) ** 2
        assert self.k > 1

    def yf(self, x):
        return 0.25 + x * self.tan

    def cf(self, x, t):
        x = np.asarray(x, float)
        out = np.where(t < x / self.k, 0.0,
                       np.where(t < x, np.exp(-self.beta / (self.k - 1.0) * (x - t)), 1.0))
        return out

    def cm(self, x, y, t):
        """Matrix concentration: region 1 above the fracture, region 2 below."""
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        above = y > self.yf(x)
        c1 = np.where(t > x, 1.0, 0.0)
        xi = (4 * y - 1) / (4 * self.tan)        # abscissa where the characteristic leaves the fracture
        below_low = y < 0.25
        c2_low = np.where(t > x, 1.0, 0.0)
        c2_mid = np.where(t > x - xi, self.cf(np.clip(xi, 0, None), t + xi - x), 0.0)
        c2 = np.where(below_low, c2_low, c2_mid)
        return np.where(above, c1, c2)


class E2:
    def __init__(self, tan1=5 / 8, tan2=1 / 4, lam_f1=200.0, lam_f3=400.0, df1=0.01, df3=0.01):
        t1, t2 = math.atan(tan1), math.atan(tan2)
        self.tan1, self.tan2 = tan1, tan2
        self.b1 = math.sin(t1) / df1
        self.k1 = lam_f1 * math.cos(t1) ** 2
        self.b2 = math.cos(t2) / df3
        self.k2 = lam_f3 * math.cos(t2) * math.sin(t2)
        self.r = lam_f3 * df3 * math.sin(t2) / (lam_f1 * df1 * math.cos(t1))
        self.x0 = (3 - tan2) / (4 * (1 + tan1 * tan2))
        self.y0 = (1 + 3 * tan1) / (4 * (1 + tan1 * tan2))
        self.r1 = self.b1 / self.k1 + self.b2 / self.k2 * tan1
        self.r2 = self.b2 / self.k2 + self.b1 / (self.k1 * tan1)
        self.c0 = (math.exp(-self.b1 / self.k1 * self.x0)
                   + self.r * math.exp(-self.b2 / self.k2 * (1 - self.y0))) / (self.r + 1)
        assert self.k1 > 1 and self.k2 * tan2 > 1

    # fractures -----------------------------------------------------------
    def cf1(self, x):
        return np.exp(-self.b1 / self.k1 * np.asarray(x, float))

    def cf4(self, y):
        return np.exp(-self.b2 / self.k2 * (1 - np.asarray(y, float)))

    def cf2(self, x):
        x = np.asarray(x, float)
        b1k1, b2k2 = self.b1 / self.k1, self.b2 / self.k2
        return np.exp(-b1k1 * x) * (self.c0 * math.exp(b1k1 * self.x0) + b1k1 / self.r1 * (
            np.exp(self.r1 * x - 3 * b2k2 / 4) - math.exp(self.r1 * self.x0 - 3 * b2k2 / 4)))

    def cf3(self, y):
        y = np.asarray(y, float)
        b1k1, b2k2 = self.b1 / self.k1, self.b2 / self.k2
        s = +b1k1 / (4 * self.tan1)   # sign fixed by the fracture ODE (see module doc)
        low = np.exp(-self.r2 / 4 + s)
        high = np.exp(-self.r2 * y + s)
        ref = math.exp(-self.r2 * self.y0 + s)
        term = np.where(y < 0.25, low, high) - ref
        return np.exp(b2k2 * y) * (self.c0 * math.exp(-b2k2 * self.y0) + b2k2 / self.r2 * term)

    # matrix ------------------------------------------------------------
    def region(self, x, y):
        above1 = y > 0.25 + x * self.tan1
        left2 = x < 0.75 - y * self.tan2
        return np.where(above1, np.where(left2, 1, 2), np.where(left2, 3, 4))

    def cm(self, x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        reg = self.region(x, y)
        xi = (y - 0.25) / self.tan1
        c3 = np.where(y < 0.25, 0.0, self.cf1(np.clip(xi, 0, None)))
        c4 = np.where(y < self.y0, self.cf3(y), self.cf2(np.clip(xi, 0, None)))
        return np.select([reg == 1, reg == 2, reg == 3, reg == 4],
                         [np.zeros_like(x), self.cf4(y), c3, c4])

    def cf_branch(self, branch, x, y):
        """Fracture concentration on branch 1..4 at points (x, y) of that branch."""
        return np.select([branch == 1, branch == 2, branch == 3, branch == 4],
                         [self.cf1(x), self.cf2(x), self.cf3(y), self.cf4(y)])


def rel_l1(weights, num, exact):
    """Relative L1 error: sum w |num - exact| / sum w |exact|."""
    return float(np.sum(weights * np.abs(num - exact)) / np.sum(weights * np.abs(exact)))
