"""Truncation of the mixed path's shell quadrature (the 1 <= s <= 2 piece of
the cubic spline, Sec. II-B / Eq. (3)), bounded by the Bernstein-ellipse
theorem for Gauss-Legendre rules.

Along an edge part at distance c from the foot line (kernel units, r0 the wall
distance), the mixed kernel integrates

    g(l) = N(U) / (S (S + r0)),  S = sqrt(l^2 + c^2),  U = 2 - S,

with N a degree-5 polynomial in U whose coefficients depend on r0 (the shell
antiderivative written in powers of U = 2 - s, so that its values near the
support's edge are small without cancellation); the term is
R0/120 * integral g dl, and the pair fraction gets -1/pi of it.  g is
analytic except at the branch points l = +-ic (and the cuts beyond them on
the imaginary axis).  Sub-intervals are at most min(0.4 q, 2 - r0) long, where
q <= S on the part (q = 1 on a shell part next to an inner part, q = c
otherwise), so every branch point lies at least 5 half-lengths from the
sub-interval: in the scaled variable the singularities are outside the
Bernstein ellipse E_rho for every rho < 5 + sqrt(26).

Theorem (Gauss-Legendre with N nodes, f analytic in E_rho, |f| <= M there):
    |I - I_N| <= (64/15) M rho^(-2N) / (1 - rho^(-2))
(Trefethen, Approximation Theory and Approximation Practice, Thm 19.3, stated
for N = n + 1 nodes).  For a sub-interval of half-length hl the bound is
multiplied by hl.  M is the maximum of |g| on the ellipse's boundary (maximum
modulus principle), evaluated on a dense set of boundary points with a 2 %
margin; the bound is minimised over rho below the singularities' ellipse.

The test takes the longest sub-intervals the rule allows at positions along
every shell part of a grid of (r0, c), checks that the 4-point rule's actual
error (against adaptive quadrature) is below the bound, and that the bound in
units of the pair fraction stays below 1e-8 per sub-interval: far below the
1e-5 per-cell tolerance even for the largest sub-interval counts per pair
(at most 64 per edge).  The per-pair kernels (the other work distributions)
use an 8-point rule on sub-intervals of at most 0.8 q, checked the same way.  The integrand's correctness is covered by the GPU
parity tests; this test is about the rule.
"""
import numpy as np
import pytest
from scipy.integrate import quad

GL4_X = np.array([0.3399810435848563, 0.8611363115940526, -0.3399810435848563, -0.8611363115940526])
GL4_W = np.array([0.6521451548625461, 0.3478548451374538, 0.6521451548625461, 0.3478548451374538])


def shell_integrand(l, r0, c):
    S = np.sqrt(l * l + c * c)
    U = 2.0 - S
    V = 2.0 - r0
    t = (r0 + 1.0) * r0
    a0 = (r0 + 1.0) * (r0 * V ** 4 + V ** 5)
    num = ((((-r0 * U + t) * U + t * V) * U + t * V ** 2) * U + t * V ** 3) * U + a0
    return num / (S * (S + r0))


_X8 = np.array([0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363])
_W8 = np.array([0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763])
GL8_X = np.concatenate([_X8, -_X8])
GL8_W = np.concatenate([_W8, _W8])


def gl4(a, b, r0, c):
    mid, hl = 0.5 * (a + b), 0.5 * (b - a)
    return hl * np.sum(GL4_W * shell_integrand(mid + hl * GL4_X, r0, c))


def gl8(a, b, r0, c):
    mid, hl = 0.5 * (a + b), 0.5 * (b - a)
    return hl * np.sum(GL8_W * shell_integrand(mid + hl * GL8_X, r0, c))


def bernstein_bound(a, b, r0, c, n_nodes=4):
    mid, hl = 0.5 * (a + b), 0.5 * (b - a)
    zs = (1j * c - mid) / hl  # the branch point in the scaled variable
    w = zs + np.sqrt(zs - 1 + 0j) * np.sqrt(zs + 1 + 0j)
    rho_s = max(abs(w), 1.0 / abs(w))
    th = np.linspace(0.0, 2.0 * np.pi, 2048, endpoint=False)
    best = np.inf
    for rho in np.geomspace(1.2, rho_s * 0.98, 48):
        z = 0.5 * (rho * np.exp(1j * th) + np.exp(-1j * th) / rho)
        M = 1.02 * np.abs(shell_integrand((mid + hl * z).astype(complex), r0, c)).max()
        best = min(best, (64.0 / 15.0) * hl * M * rho ** (-2 * n_nodes) / (1.0 - rho ** -2))
    return best, rho_s


def _rounding(a, b, r0, c):
    """FP64 rounding allowance of a rule's value: the integrand's polynomial cancels near r0 = 2, so its
    relative rounding grows there; 1e-11 of the integral of |g| covers it."""
    ll = np.linspace(a, b, 33)
    return 1e-11 * (b - a) * np.abs(shell_integrand(ll, r0, c)).max()


def _cases(rule):
    """Longest sub-intervals of the longest shell part (from l1, or from -l2 when there is no inner part and the
    part straddles l = 0, to l2), at several positions, with the kernels' sub-interval counts and caps."""
    out = []
    for r0 in (0.0, 0.05, 0.4, 0.9, 1.3, 1.7, 1.95, 1.99, 1.999):
        for c in np.linspace(max(r0, 0.02), 1.9999, 9):
            inner = c < 1.0
            l2 = np.sqrt(4.0 - c * c)
            l1 = np.sqrt(1.0 - c * c) if inner else 0.0
            q = 1.0 if inner else c
            lo = l1 if inner else -l2
            part = l2 - lo
            if part <= 0:
                continue
            if rule == 4:  # the task-batch kernel: at most min(0.4 q, 2 - r0), at most 32 per part
                n = min(max(int(np.ceil(part / min(0.4 * q, 2.0 - r0))), 1), 32)
            else:  # the per-pair kernels: at most 0.8 q, at most 8 per part
                n = min(max(int(np.ceil(part / (0.8 * q))), 1), 8)
            L = part / n
            for a in np.linspace(lo, l2 - L, 4):
                out.append((r0, float(c), float(a), float(L)))
    return out


CASES = _cases(4)
CASES8 = _cases(8)


def test_singularities_outside_rule_ellipse():
    """The length rule keeps the branch points outside E_rho for rho up to 5 + sqrt(26) (the caps on the
    sub-interval count never lengthen a sub-interval past 0.4 q)."""
    for r0, c, a, L in CASES:
        _, rho_s = bernstein_bound(a, a + L, r0, c)
        assert rho_s >= 5.0 + np.sqrt(26.0) - 1e-9, (r0, c, a, L, rho_s)


@pytest.mark.parametrize("chunk", range(4))
def test_gl4_truncation_within_bernstein_bound(chunk):
    worst = 0.0
    for r0, c, a, L in CASES[chunk::4]:
        b = a + L
        ref = quad(lambda l: shell_integrand(l, r0, c), a, b, epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        err = abs(gl4(a, b, r0, c) - ref)
        bound, _ = bernstein_bound(a, b, r0, c)
        assert err <= bound + _rounding(a, b, r0, c), (r0, c, a, L, err, bound)
        R0 = np.sqrt(max(c * c - r0 * r0, 0.0))
        frac_bound = bound * R0 / (120.0 * np.pi)
        assert frac_bound <= 1e-8, (r0, c, a, L, frac_bound)
        worst = max(worst, frac_bound)
    assert worst > 0.0


@pytest.mark.parametrize("chunk", range(2))
def test_gl8_truncation_within_bernstein_bound(chunk):
    """The 8-point rule of the per-pair kernels (distributions 0-2), sub-intervals up to 0.8 q: the branch points
    stay outside E_rho for rho < 2.5 + sqrt(7.25)."""
    for r0, c, a, L in CASES8[chunk::2]:
        b = a + L
        ref = quad(lambda l: shell_integrand(l, r0, c), a, b, epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        err = abs(gl8(a, b, r0, c) - ref)
        bound, rho_s = bernstein_bound(a, b, r0, c, n_nodes=8)
        assert rho_s >= 2.5 + np.sqrt(7.25) - 1e-9
        assert err <= bound + _rounding(a, b, r0, c), (r0, c, a, L, err, bound)
        R0 = np.sqrt(max(c * c - r0 * r0, 0.0))
        assert bound * R0 / (120.0 * np.pi) <= 1e-8, (r0, c, a, L, bound)
