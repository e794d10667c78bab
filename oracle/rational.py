"""Rational approximation of x^(-1/2) for the heatbath (Sec. IV B).

Test infrastructure only: see the package docstring.

The heatbath needs the coefficients of a rational function of the form of
eqn rat_approx,

    f(x) = alpha_0 + sum_k alpha_k / (beta_k + x),

close to x^(-1/2) on the spectrum of M_EOFA. The paper takes them from a
Remez fit on measured spectral bounds and prints none; they are an input of
the heatbath on both sides of every test. Here they come from a closed-form
construction instead: Gauss-Legendre quadrature of

    x^(-1/2) = (2/pi) int_0^inf dt / (t^2 + x),

after the substitution t = sqrt(c) tan(theta), theta in (0, pi/2):

    x^(-1/2) = (2 sqrt(c) / pi) int_0^(pi/2) dtheta / (cos^2(theta) (x + c tan^2(theta))).

Every node theta_j with weight w_j gives one pole,

    beta_j = c tan^2(theta_j),   alpha_j = 2 sqrt(c) w_j / (pi cos^2(theta_j)),   alpha_0 = 0,

all beta_j > 0 and all alpha_j > 0, so f(x) > 0 on x > 0. At x = c the
integrand is the constant 1/sqrt(c), which the rule integrates exactly;
c = sqrt(lmin * lmax) centres the rule on [lmin, lmax] in log x, where the
error then falls off exponentially with the number of nodes.
"""
import numpy as np


def inv_sqrt_coefficients(lmin, lmax, n_poles):
    """(alpha[0..n], beta[0..n-1]) of f(x) = alpha_0 + sum alpha_k / (beta_k + x)."""
    if not (0.0 < lmin <= lmax) or n_poles < 1:
        raise ValueError("need 0 < lmin <= lmax and n_poles >= 1")
    c = np.sqrt(lmin * lmax)
    nodes, weights = np.polynomial.legendre.leggauss(n_poles)
    theta = 0.25 * np.pi * (nodes + 1.0)   # [-1, 1] -> [0, pi/2]
    w = 0.25 * np.pi * weights
    cos2 = np.cos(theta) ** 2
    beta = c * np.tan(theta) ** 2
    alpha = 2.0 * np.sqrt(c) * w / (np.pi * cos2)
    return np.concatenate([[0.0], alpha]), beta


def evaluate(alpha, beta, x):
    """f(x) for scalar or array x."""
    x = np.asarray(x, dtype=np.float64)
    out = np.full(x.shape, float(alpha[0]))
    for a, b in zip(alpha[1:], beta):
        out = out + a / (b + x)
    return out


def max_rel_error(alpha, beta, lmin, lmax, n=20001):
    """max over [lmin, lmax] (geometric grid) of |1 - sqrt(x) f(x)|."""
    x = np.geomspace(lmin, lmax, n)
    return float(np.max(np.abs(1.0 - np.sqrt(x) * evaluate(alpha, beta, x))))


def heatbath_eps_bound(alpha, beta, eigenvalues):
    """max over the given eigenvalues lam of |1 - lam f(lam)^2|: the largest
    eps (eqn heatbath_rel_err) that phi = f(M) eta can give for exact solves,
    since eta^dag eta - phi^dag M phi = eta^dag (1 - M f(M)^2) eta."""
    lam = np.asarray(eigenvalues, dtype=np.float64)
    return float(np.max(np.abs(1.0 - lam * evaluate(alpha, beta, lam) ** 2)))
