"""Exact Gaussian-rational brute force for tiny precoding problems.

TEST INFRASTRUCTURE ONLY (pins the FP64 oracle; never used by the product).

With a Gaussian-integer channel, Gaussian-integer symbols and a rational
regularizer every quantity of the WF precoder is a Gaussian rational except
the final square root of the precoding factor.  So the squared factor
beta^2 and the unnormalized output beta * x are computed here exactly, with
Python ``fractions`` and Gauss-Jordan elimination (not Cholesky), straight
from the definitions:

* Theorem 1 (centralized WF): Q = (H_dl^H H_dl + kappa I_B)^-1 H_dl^H and
  beta^2 = tr(Q^H Q) Es / rho^2 -- the B x B form, no Lemma 1, no
  push-through identity.  In the B x U storage convention of this project
  H_dl^H = H, so Q = (H H^H + kappa I_B)^-1 H.
* ZF: the pseudo-inverse precoder (kappa = 0), U x U Gram form.
* Sec. III-C (FD): per cluster rho_c^2 = rho^2 / C, kappa_c = tau C kappa,
  Q_c from the B_c x B_c form when B_c < U and from the U x U form
  otherwise, weight^2 = rho_c^2 / (tr(Q_c^H Q_c) Es).
"""
from __future__ import annotations

from fractions import Fraction as F


class GQ:
    """Gaussian rational re + i im with Fraction parts."""

    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = F(re)
        self.im = F(im)

    def __add__(self, o):
        o = _g(o)
        return GQ(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _g(o)
        return GQ(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _g(o) - self

    def __mul__(self, o):
        o = _g(o)
        return GQ(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = _g(o)
        den = o.re * o.re + o.im * o.im
        num = self * o.conj()
        return GQ(num.re / den, num.im / den)

    def __neg__(self):
        return GQ(-self.re, -self.im)

    def conj(self):
        return GQ(self.re, -self.im)

    def abs2(self):
        return self.re * self.re + self.im * self.im

    def is_zero(self):
        return self.re == 0 and self.im == 0

    def __complex__(self):
        return complex(float(self.re), float(self.im))


def _g(v):
    if isinstance(v, GQ):
        return v
    if isinstance(v, complex):
        return GQ(F(v.real), F(v.imag))
    return GQ(v, 0)


def mat(rows):
    return [[_g(v) for v in r] for r in rows]


def matmul(A, B):
    n, m, p = len(A), len(B), len(B[0])
    return [[sum((A[i][k] * B[k][j] for k in range(m)), GQ()) for j in range(p)] for i in range(n)]


def herm(A):
    return [[A[i][j].conj() for i in range(len(A))] for j in range(len(A[0]))]


def inverse(A):
    """Gauss-Jordan elimination with exact pivot search (nonzero pivot)."""
    n = len(A)
    M = [[A[i][j] for j in range(n)] + [GQ(1 if i == j else 0) for j in range(n)] for i in range(n)]
    for col in range(n):
        piv = next((r for r in range(col, n) if not M[r][col].is_zero()), None)
        if piv is None:
            raise ZeroDivisionError("singular")
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [v / p for v in M[col]]
        for r in range(n):
            if r != col and not M[r][col].is_zero():
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [row[n:] for row in M]


def _add_diag(A, kappa):
    return [[A[i][j] + (kappa if i == j else 0) for j in range(len(A))] for i in range(len(A))]


def frob2(A):
    return sum((v.abs2() for r in A for v in r), F(0))


def central_wf(H, s_list, kappa, power=1, Es=1):
    """Theorem 1, B x B form.  H: B x U (list of lists of ints/complex),
    s_list: list of length-U symbol vectors.  Returns (beta^2, [beta*x])."""
    H = mat(H)
    B = len(H)
    kappa = F(kappa)
    Q = matmul(inverse(_add_diag(matmul(H, herm(H)), kappa)), H)  # B x U
    beta2 = frob2(Q) * F(Es) / F(power)
    outs = []
    for s in s_list:
        sv = [[_g(v)] for v in s]
        outs.append([r[0] for r in matmul(Q, sv)])
    return beta2, outs


def central_zf(H, s_list, power=1, Es=1):
    """Zero-forcing: the kappa = 0 case of Theorem 1 taken as the textbook
    pseudo-inverse precoder Q = H_dl^H (H_dl H_dl^H)^-1 (U <= B, full rank);
    in this project's convention Q = H (H^H H)^-1.  Returns (beta^2, [beta*x])."""
    H = mat(H)
    Q = matmul(H, inverse(matmul(herm(H), H)))  # B x U
    beta2 = frob2(Q) * F(Es) / F(power)
    outs = []
    for s in s_list:
        sv = [[_g(v)] for v in s]
        outs.append([r[0] for r in matmul(Q, sv)])
    return beta2, outs


def fd_wf(H, s_list, kappa, sizes, tau, power=1, Es=1, zf=False):
    """Sec. III-C.  Returns ([w_c^2], [x_c / w_c concatenated per symbol])."""
    H = mat(H)
    U = len(H[0])
    C = len(sizes)
    rho_c2 = F(power) / C
    kappa_c = F(0) if zf else F(tau) * C * F(kappa)
    w2 = []
    per_sym = [[] for _ in s_list]
    row0 = 0
    for Bc in sizes:
        Hc = H[row0:row0 + Bc]
        if Bc < U:
            Q = matmul(inverse(_add_diag(matmul(Hc, herm(Hc)), kappa_c)), Hc)
        else:
            Q = matmul(Hc, inverse(_add_diag(matmul(herm(Hc), Hc), kappa_c)))
        w2.append(rho_c2 / (frob2(Q) * F(Es)))
        for k, s in enumerate(s_list):
            sv = [[_g(v)] for v in s]
            per_sym[k].extend(r[0] for r in matmul(Q, sv))
        row0 += Bc
    return w2, per_sym
