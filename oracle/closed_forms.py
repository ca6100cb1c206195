"""Textbook closed forms used as pins of the simulation (oracle side).

* Vasicek (1977) zero-coupon bond, Brigo & Mercurio (2006) eq. (3.8):
      P(t, t+tau) = exp(lnA(tau) - B(tau) r_t),
      B(tau)   = (1 - exp(-a tau)) / a,
      lnA(tau) = (b - sigma^2 / (2 a^2)) (B(tau) - tau) - sigma^2 B(tau)^2 / (4 a).
  The paper states (Appendix B, footnote on the swap price) that the zero-coupon
  price has a closed form under the affine short-rate model without printing it.
* Ornstein-Uhlenbeck moments of r_t.
* CIR survival E[exp(-int_0^t gamma)] (Cox, Ingersoll & Ross 1985):
      h = sqrt(kappa^2 + 2 nu^2),
      B = 2 (e^{ht} - 1) / (2h + (kappa + h)(e^{ht} - 1)),
      A = [2h e^{(kappa+h)t/2} / (2h + (kappa + h)(e^{ht} - 1))]^{2 kappa theta / nu^2},
      S(t) = A exp(-B lambda0).
"""
from __future__ import annotations

import numpy as np


def vasicek_B(a, tau):
    return (1.0 - np.exp(-a * tau)) / a


def vasicek_lnA(a, b, sigma, tau):
    B = vasicek_B(a, tau)
    return (b - sigma ** 2 / (2.0 * a ** 2)) * (B - tau) - sigma ** 2 * B ** 2 / (4.0 * a)


def vasicek_zc(a, b, sigma, r, tau):
    """Price at t of the zero-coupon bond maturing at t + tau, given r_t."""
    return np.exp(vasicek_lnA(a, b, sigma, tau) - vasicek_B(a, tau) * r)


def ou_mean(a, b, r0, t):
    return b + (r0 - b) * np.exp(-a * t)


def ou_var(a, sigma, t):
    return sigma ** 2 * (1.0 - np.exp(-2.0 * a * t)) / (2.0 * a)


def cir_survival(kappa, theta, nu, lam0, t):
    h = np.sqrt(kappa ** 2 + 2.0 * nu ** 2)
    e = np.expm1(h * t)
    den = 2.0 * h + (kappa + h) * e
    B = 2.0 * e / den
    A = (2.0 * h * np.exp((kappa + h) * t / 2.0) / den) ** (2.0 * kappa * theta / nu ** 2)
    return A * np.exp(-B * lam0)
