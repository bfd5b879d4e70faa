"""Keldysh photoionization rate in FP64, evaluated in situ (paper Sec. 2.1).

TEST INFRASTRUCTURE (part of the oracle).  Follows Sec. 2.1 of the paper:

* Keldysh parameter  gamma = omega sqrt(m* Delta) / (e E)   (Sec. 2.1, text)
* gamma1 = gamma^2/(1+gamma^2), gamma2 = 1/(1+gamma^2)      (Sec. 2.1, text)
* effective gap x, Eq. (1)
* rate W [m^-3 s^-1], Eq. (2), with the series Q(gamma, x) of Eq. (3),
  truncated after its first 500 terms (Sec. 2.1, paragraph after Eq. (3)).

Readings (where the paper is silent):
* The elliptic integrals take the *parameter* m = k^2 (so kappa(gamma1) is
  K(m = gamma1)); gamma1 and gamma2 are the squares of Keldysh's moduli.
* floor(x + 1) is the integer part of x plus one.
* The leading factor 2 of Eq. (2) is kept as printed.

Numerics: kappa and epsilon are computed by the arithmetic-geometric mean
(Abramowitz & Stegun 17.6) from both the parameter and its complement, each
formed directly (never as 1 - other), so small fields (gamma1 -> 1) keep full
precision.  The Dawson integral uses Rybicki's exponentially convergent sum
(G. B. Rybicki, Computers in Physics 3, 85 (1989)) with step h = 0.2, and its
Maclaurin series near zero.

Pins (tests/test_oracle_keldysh.py): K, E against scipy and the Legendre
relation; Dawson against scipy and its ODE; W against the multiphoton and
tunneling limits of the formula and against its truncation bound.
"""

import numpy as np

from .constants import C, QE, ME, HBAR

_SQRT_PI_INV = 1.0 / np.sqrt(np.pi)
_RYB_C = {k: np.exp(-(k * 0.2) ** 2) for k in range(1, 35, 2)}
_DAWSON_MAX = 0.5410442246      # max of the Dawson integral (at z = 0.9241)


def ellip_KE(m, m1):
    """Complete elliptic integrals K(m), E(m) for parameter m with m1 = 1 - m.

    Both ``m`` and ``m1`` are passed so that neither is formed by cancellation.
    A&S 17.6: a0 = 1, b0 = sqrt(m1), c0 = sqrt(m);
    K = pi / (2 a_inf),  E = K (1 - sum_n 2^(n-1) c_n^2).
    """
    m = np.asarray(m, dtype=np.float64)
    m1 = np.asarray(m1, dtype=np.float64)
    a = np.ones_like(m)
    b = np.sqrt(m1)
    s = 0.5 * m            # n = 0 term: 2^-1 c0^2
    p = 1.0                # 2^(n-1) for n = 1
    for _ in range(64):
        c = 0.5 * (a - b)
        a, b = 0.5 * (a + b), np.sqrt(a * b)
        s = s + p * c * c
        p *= 2.0
        if np.all(np.abs(c) <= 4e-16 * a):    # converged to within rounding
            break
    K = np.pi / (2.0 * a)
    return K, K * (1.0 - s)


def dawson(z):
    """Dawson integral F(z) = exp(-z^2) int_0^z exp(t^2) dt, FP64, vectorised."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    az = np.abs(z)
    small = az < 0.2
    if np.any(small):
        x = z[small]
        x2 = x * x
        # Maclaurin series: sum_k (-1)^k 2^k x^(2k+1) / (2k+1)!!
        term = x.copy()
        acc = x.copy()
        for k in range(1, 14):
            term = term * (-2.0 * x2) / (2 * k + 1)
            acc = acc + term
        out[small] = acc
    big = ~small
    if np.any(big):
        h = 0.2
        x = az[big]
        n0 = 2.0 * np.rint(0.5 * x / h)
        xp = x - n0 * h
        e1 = np.exp(2.0 * xp * h)        # exp(2 xp k h) advanced by e1^2 per odd k
        e2 = e1 * e1
        ek = e1.copy()
        acc = np.zeros_like(x)
        for k in range(1, 35, 2):
            acc = acc + _RYB_C[k] * (ek / (n0 + k) + 1.0 / (ek * (n0 - k)))
            ek = ek * e2
        out[big] = np.sign(z[big]) * _SQRT_PI_INV * np.exp(-xp * xp) * acc
    return out


def keldysh_parts(A, gap_eV, mred, lam):
    """Intermediate quantities of Eq. (1)-(3) at field amplitude A [V/m].

    Returns dict with gamma, gamma1, gamma2, K1=kappa(gamma1), E1=eps(gamma1),
    K2=kappa(gamma2), E2=eps(gamma2), x (Eq. 1), N = floor(x+1), alpha (the
    per-term decay exponent of Eq. 3), beta (the Dawson-argument scale of Eq. 3),
    prefactor (Eq. 2 without Q and the exponential).
    """
    A = np.asarray(A, dtype=np.float64)
    omega = 2.0 * np.pi * C / lam
    Delta = gap_eV * QE
    mstar = mred * ME
    gamma = omega * np.sqrt(mstar * Delta) / (QE * A)
    g2sq = gamma * gamma
    gamma2 = 1.0 / (1.0 + g2sq)
    gamma1 = g2sq / (1.0 + g2sq)
    K1, E1 = ellip_KE(gamma1, gamma2)
    K2, E2 = ellip_KE(gamma2, gamma1)
    x = (2.0 / np.pi) * (Delta / (HBAR * omega)) * E2 / np.sqrt(gamma1)
    N = np.floor(x + 1.0)
    alpha = np.pi * (K1 - E1) / E2
    beta = np.pi ** 2 / (2.0 * K2 * E2)
    pref = 2.0 * (2.0 * omega / (9.0 * np.pi)) * (mstar * omega / (HBAR * np.sqrt(gamma1))) ** 1.5
    return dict(gamma=gamma, gamma1=gamma1, gamma2=gamma2, K1=K1, E1=E1, K2=K2,
                E2=E2, x=x, N=N, alpha=alpha, beta=beta, pref=pref, omega=omega)


def keldysh_rate(A, gap_eV, mred, lam, terms=500, N_override=None, tol_bits=60):
    """Keldysh volumetric ionization rate W(A) [m^-3 s^-1], Eq. (2)-(3).

    ``terms``: at most the series terms n = 0 .. terms-1 (the paper uses 500).
    ``tol_bits``: the sum stops after term n once the bound of the remaining
    tail, max(Dawson) e^{-(n+1) alpha} / (1 - e^{-alpha}), is below 2^-tol_bits
    of the partial sum (the adaptive tolerance the paper names as future work;
    60 leaves the FP64 result of the full sum).
    ``N_override``: evaluate with floor(x+1) replaced by a given integer (the
    analytic continuation of one channel; used only by tests).
    """
    A = np.atleast_1d(np.asarray(A, dtype=np.float64))
    p = keldysh_parts(A, gap_eV, mred, lam)
    N = p["N"] if N_override is None else np.full_like(A, float(N_override))
    d = N - p["x"]
    alpha, beta = p["alpha"], p["beta"]
    Q = np.zeros_like(A)
    live = np.arange(len(A))
    tol = 2.0 ** -int(tol_bits)
    chunk = 8
    for n_lo in range(0, terms, chunk):
        n = np.arange(n_lo, min(terms, n_lo + chunk), dtype=np.float64)[None, :]
        a_l = alpha[live][:, None]
        arg = np.sqrt(np.maximum(beta[live][:, None] * (d[live][:, None] + n), 0.0))
        # partial sums after each term of the chunk, and the tail bound after it
        S = Q[live][:, None] + np.cumsum(np.exp(-n * a_l) * dawson(arg), axis=1)
        tail = _DAWSON_MAX * np.exp(-(n + 1.0) * a_l) / (-np.expm1(-a_l))
        stop = tail < tol * S
        first = np.where(stop.any(axis=1), stop.argmax(axis=1), S.shape[1] - 1)
        Q[live] = S[np.arange(len(live)), first]
        live = live[~stop.any(axis=1)]
        if len(live) == 0:
            break
    Q *= np.sqrt(np.pi / (2.0 * p["K2"]))
    return p["pref"] * Q * np.exp(-N * p["alpha"])


def ponderomotive_eV(I_Wcm2, me_star, lam):
    """Ponderomotive energy U_p = e^2 E0^2 / (4 m omega^2) for linear polarisation,
    with I = (1/2) c eps0 E0^2 (the convention Sec. 5's U_p values pin)."""
    from .constants import EPS0
    E0 = np.sqrt(2.0 * I_Wcm2 * 1e4 / (C * EPS0))
    omega = 2.0 * np.pi * C / lam
    return QE ** 2 * E0 ** 2 / (4.0 * me_star * ME * omega ** 2) / QE
