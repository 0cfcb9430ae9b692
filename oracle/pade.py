"""Pade coefficients of the split-step propagator, in high precision (mpmath).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle.  Only tests/, the smoke check and the
benchmark's CPU-baseline leg may import it; the product library never does.

What is computed (Sec. 2, the SSP Pade form and its coefficient definition; Algorithm 1,
first step):  the [p/p] Pade approximant R(x) = P(x)/Q(x) of

        f(x) = exp(i sigma (sqrt(1 + x) - 1)),     sigma = k0 * dr,

so that the range step is exp(i dr sqrt(d_z^2 + k^2)) ~ e^{i k0 dr} R(X) with
X = (d_z^2 + k^2 - k0^2)/k0^2.  The sum (partial-fraction) form used by the paper is
R(x) = d0 + sum_j d_j / (1 + b_j x); the equivalent product form is
R(x) = C prod_j (1 + a_j x) / (1 + b_j x).

Steps, in the order a textbook Pade construction takes them:
  1. Taylor coefficients f_n of f about x = 0 up to n = 2p, from f' = g' f with
     g(x) = i sigma (sqrt(1+x) - 1), i.e. n f_n = sum_{k=1..n} k g_k f_{n-k},
     g_k = i sigma * binom(1/2, k).
  2. Denominator Q(x) = sum q_i x^i, q_0 = 1, from the linear conditions
     sum_{i=0..p} q_i f_{n-i} = 0, n = p+1..2p (the Pade matching conditions).
  3. Numerator P_n = sum_{i=0..min(n,p)} q_i f_{n-i}, n = 0..p.
  4. Roots r_j of Q give b_j = -1/r_j; roots s_j of P give a_j = -1/s_j.
  5. Sum form: d0 = lim_{x->inf} R = C prod a_j / b_j and residues
     d_j = C prod_i (1 - a_i/b_j) / prod_{i != j} (1 - b_i/b_j).

Rotated branch cut (a reading: the paper does not define rotation): the Pade approximant
is taken of F(Z) = exp(i sigma (e^{i alpha/2} sqrt(1+Z) - 1)) in Z = e^{-i alpha}(1+x) - 1,
and each factor 1 + b~ Z is mapped back to (1 + b~ beta)(1 + b x) with beta = e^{-i alpha}-1,
b = b~ e^{-i alpha} / (1 + b~ beta).  alpha = 0 is the standard approximant.

Factor order (a reading; the paper leaves it free): ascending arg(b_j), ties by |b_j|.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import mpmath as mp
import numpy as np

DPS = 60


@dataclass
class PadeCoeffs:
    sigma: float
    order: int
    alpha: float
    b: np.ndarray          # complex128 [p]   denominator coefficients (sorted)
    a: np.ndarray          # complex128 [p]   numerator coefficients paired with b
    C: complex             # product-form constant (1 for the standard approximant)
    d0: complex            # sum-form constant term
    d: np.ndarray          # complex128 [p]   sum-form residues paired with b
    taylor: List[complex]  # f_0..f_2p (as Python complex), for reference

    def R(self, x):
        """Evaluate R(x) = d0 + sum d_j/(1 + b_j x) in FP64 (numpy broadcasting)."""
        x = np.asarray(x, dtype=np.complex128)
        out = np.full(x.shape, self.d0, dtype=np.complex128)
        for dj, bj in zip(self.d, self.b):
            out = out + dj / (1.0 + bj * x)
        return out

    def R_product(self, x):
        x = np.asarray(x, dtype=np.complex128)
        out = np.full(x.shape, self.C, dtype=np.complex128)
        for aj, bj in zip(self.a, self.b):
            out = out * (1.0 + aj * x) / (1.0 + bj * x)
        return out


def taylor_coefficients(sigma, n, alpha=0.0):
    """f_0..f_n of F(Z) = exp(i sigma (e^{i alpha/2} sqrt(1+Z) - 1)) as mpc (alpha=0 gives
    the standard f)."""
    with mp.workdps(DPS):
        s = mp.mpf(sigma)
        rot = mp.expj(mp.mpf(alpha) / 2)
        g = [1j * s * (rot - 1)] + [1j * s * rot * mp.binomial(mp.mpf(1) / 2, k)
                                    for k in range(1, n + 1)]
        f = [mp.exp(g[0])]
        for m in range(1, n + 1):
            acc = mp.mpc(0)
            for k in range(1, m + 1):
                acc += k * g[k] * f[m - k]
            f.append(acc / m)
        return f


def _sort_key(bj):
    return (float(mp.arg(bj)), float(abs(bj)))


def pade(sigma: float, order: int, alpha: float = 0.0) -> PadeCoeffs:
    """[p/p] Pade coefficients (see module docstring)."""
    p = int(order)
    if p < 1:
        raise ValueError("order must be >= 1")
    with mp.workdps(DPS):
        f = taylor_coefficients(sigma, 2 * p, alpha)
        # step 2: q_1..q_p from sum_{i=0..p} q_i f_{n-i} = 0, n = p+1..2p
        A = mp.matrix(p, p)
        rhs = mp.matrix(p, 1)
        for row, n in enumerate(range(p + 1, 2 * p + 1)):
            for i in range(1, p + 1):
                A[row, i - 1] = f[n - i]
            rhs[row] = -f[n]
        qs = mp.lu_solve(A, rhs)
        q = [mp.mpc(1)] + [qs[i] for i in range(p)]
        # step 3: numerator
        P = [sum(q[i] * f[n - i] for i in range(0, min(n, p) + 1)) for n in range(p + 1)]
        # step 4: roots (polyroots wants the highest power first)
        rq = mp.polyroots(list(reversed(q)), maxsteps=400, extraprec=4 * DPS)
        rp = mp.polyroots([c / P[0] for c in reversed(P)], maxsteps=400, extraprec=4 * DPS)
        bt = [-1 / r for r in rq]
        at = [-1 / s for s in rp]
        Ct = P[0]                      # P(Z) = P_0 prod (1 + a~ Z), Q(Z) = prod (1 + b~ Z)
        # pair each numerator factor with a denominator factor: a_j = conj(b_j) holds for
        # the standard approximant; for the rotated one pair by the same rule in Z.
        bt.sort(key=_sort_key)
        paired = []
        pool = list(at)
        for bj in bt:
            k = min(range(len(pool)), key=lambda i: abs(pool[i] - mp.conj(bj)))
            paired.append(pool.pop(k))
        at = paired
        if alpha != 0.0:
            beta = mp.expj(-mp.mpf(alpha)) - 1
            gam = mp.expj(-mp.mpf(alpha))
            C = Ct
            b, a = [], []
            for bj, aj in zip(bt, at):
                C = C * (1 + aj * beta) / (1 + bj * beta)
                b.append(bj * gam / (1 + bj * beta))
                a.append(aj * gam / (1 + aj * beta))
        else:
            C, b, a = Ct, bt, at
        # order the x-space factors by the same rule
        idx = sorted(range(p), key=lambda j: _sort_key(b[j]))
        b = [b[j] for j in idx]
        a = [a[j] for j in idx]
        # step 5: sum form from the product form
        d0 = C
        for aj, bj in zip(a, b):
            d0 = d0 * aj / bj
        d = []
        for j in range(p):
            num = C
            for i in range(p):
                num = num * (1 - a[i] / b[j])
            den = mp.mpc(1)
            for i in range(p):
                if i != j:
                    den = den * (1 - b[i] / b[j])
            d.append(num / den)
        cc = lambda v: complex(v)
        return PadeCoeffs(sigma=float(sigma), order=p, alpha=float(alpha),
                          b=np.array([cc(v) for v in b]), a=np.array([cc(v) for v in a]),
                          C=cc(C), d0=cc(d0), d=np.array([cc(v) for v in d]),
                          taylor=[cc(v) for v in f])
