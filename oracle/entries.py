"""Matrix entries by three-term recurrences, float64.

Test infrastructure only (see ``oracle/__init__``).

* Chebyshev T_m(x_j) = cos(m theta_j) at Chebyshev-Gauss nodes, eq. (cheb_matrix);
  theta_j = pi (2j+1) / (2N), so m theta_j = pi q / (2N) with the integer
  q = m (2j+1) mod 4N, which keeps the angle exact for large m.  The other
  trigonometric generators, sin(m theta_j) (sec. 2) and cos(m theta_j)^s
  (eq. cosd2), use the same angle.
* Orthonormal Jacobi polynomials p_m^{(alpha,beta)} (the matrix of eq. (Jac_matrix)
  normalised as in sec. 5.2): x p_m = a_{m+1} p_{m+1} + b_m p_m + a_m p_{m-1}
  with the textbook coefficients (DLMF 18.9.2, 18.2.11), p_0 = mu0^{-1/2}.
* Laguerre functions l_m(x) = exp(-x/2) L_m(x) (sec. 4):
  (m+1) l_{m+1} = (2m+1-x) l_m - m l_{m-1}, l_0 = exp(-x/2).
* Hermite functions psi_m(x) = exp(-x^2/2) h_m(x), h_m orthonormal for exp(-x^2):
  psi_{m+1} = sqrt(2/(m+1)) x psi_m - sqrt(m/(m+1)) psi_{m-1},
  psi_0 = pi^{-1/4} exp(-x^2/2).

The exponential factors of the two function families under- and overflow at
large nodes (exp(-x/2) < 1e-308 for x > 1417), so those recurrences carry each
row as mantissa * 2^E with an integer E, rescale the mantissas by an exact
power of two whenever they grow past 2^500, and form mantissa * 2^E only when a
value is stored.
"""

import math

import mpmath
import numpy as np

_RESCALE = 2.0 ** -500
_BIG = 2.0 ** 500

# ln 2 split so that n * LN2_HI is exact for |n| < 2^21 (Cody-Waite reduction)
LN2_HI = float(round(math.log(2.0) * 2.0 ** 32)) / 2.0 ** 32
mpmath.mp.dps = 40
LN2_LO = float(mpmath.log(2) - mpmath.mpf(LN2_HI))


def exp_neg_scaled(a):
    """exp(-a) = mant * 2^E for a >= 0, with mant in [0.7, 1.42] and integer E."""
    a = np.asarray(a, dtype=np.float64)
    n = np.rint(a / math.log(2.0))
    r = (a - n * LN2_HI) - n * LN2_LO
    return np.exp(-r), (-n).astype(np.int64)


def exact_square(x):
    """x*x = hi + lo exactly (Veltkamp/Dekker splitting)."""
    x = np.asarray(x, dtype=np.float64)
    c = 134217729.0 * x  # 2^27 + 1
    xh = c - (c - x)
    xl = x - xh
    hi = x * x
    lo = ((xh * xh - hi) + 2.0 * xh * xl) + xl * xl
    return hi, lo


# --------------------------------------------------------------------------- Chebyshev

def chebyshev_t(j, N, m0, m1):
    """cos(m theta_j), rows j (Chebyshev-Gauss node indices), columns m0 .. m1-1."""
    j = np.asarray(j, dtype=np.int64)
    m = np.arange(m0, m1, dtype=np.int64)
    q = np.mod(np.outer(2 * j + 1, m), 4 * N)
    return np.cos(np.pi * q.astype(np.float64) / (2.0 * N))


def sine(j, N, m0, m1):
    """sin(m theta_j) at the Chebyshev-Gauss angles: the sine generator that
    Algorithms 1 and 2 compress as they do the cosine one (sec. 2, after
    Algorithm 2); the same exact angle as chebyshev_t."""
    j = np.asarray(j, dtype=np.int64)
    m = np.arange(m0, m1, dtype=np.int64)
    q = np.mod(np.outer(2 * j + 1, m), 4 * N)
    return np.sin(np.pi * q.astype(np.float64) / (2.0 * N))


def cos_power(j, N, m0, m1, s):
    """cos(m theta_j)^s, eq. (cosd2) (s = 2, 3, 4, 5), at the Chebyshev-Gauss angles."""
    return chebyshev_t(j, N, m0, m1) ** int(s)


def cexp(j, N, m0, m1):
    """exp(i m theta_j) at the Chebyshev-Gauss angles: the complex generator of
    sec. 2 (after Algorithm 2), cos + i sin at the exact angle of chebyshev_t."""
    return chebyshev_t(j, N, m0, m1) + 1j * sine(j, N, m0, m1)


# --------------------------------------------------------------------------- Laguerre, spectral domain

def laguerre_spectral_k(j, T):
    """k_j = 2 pi j / T, the wave numbers of the Fourier coefficients (sec. 4.1)."""
    return 2.0 * np.pi * np.asarray(j, dtype=np.float64) / T


def laguerre_spectral_phase(j, eta, T):
    """phi_j with (-eta/2 - i k_j) / (eta/2 - i k_j) = exp(i phi_j): the ratio
    has modulus one and equals -(eta/2 + i k)/(eta/2 - i k) = exp(i (pi + 2
    atan(2k/eta))); phi_j = 2 atan(2 k_j / eta) - pi, in [-pi, 0)."""
    return 2.0 * np.arctan(2.0 * laguerre_spectral_k(j, T) / eta) - np.pi


def laguerre_spectral(j, eta, T, m0, m1, phi=None):
    """C[j, m] = (-eta/2 - i k_j)^m / (eta/2 - i k_j)^(m+1)  (eq. main_formula2,
    the matrix of eq. lag_matrix), evaluated as exp(i m phi_j) / (eta/2 - i k_j)
    with the phase m phi_j a float64 product (rounded once).  phi: the row
    phases to use (laguerre_spectral_phase by default)."""
    j = np.asarray(j)
    k = laguerre_spectral_k(j, T)
    ph = laguerre_spectral_phase(j, eta, T) if phi is None else np.asarray(phi, dtype=np.float64)
    m = np.arange(m0, m1, dtype=np.float64)
    ang = np.outer(ph, m)
    return np.exp(1j * ang) / (0.5 * eta - 1j * k)[:, None]


# --------------------------------------------------------------------------- Jacobi

def jacobi_coefficients(n, alpha, beta):
    """Recurrence coefficients a_k (k=1..n) and b_k (k=0..n) of the orthonormal system.

    b_k = (beta^2 - alpha^2) / ((2k+ab)(2k+ab+2)),        b_0 = (beta-alpha)/(ab+2)
    a_k^2 = 4k(k+alpha)(k+beta)(k+ab) / ((2k+ab)^2 (2k+ab+1)(2k+ab-1)),
    a_1^2 = 4(1+alpha)(1+beta) / ((2+ab)^2 (3+ab))   (the k=1 limit, valid for ab=-1)
    with ab = alpha + beta.
    """
    ab = alpha + beta
    k = np.arange(n + 1, dtype=np.float64)
    b = np.empty(n + 1)
    b[0] = (beta - alpha) / (ab + 2.0)
    kk = k[1:]
    b[1:] = (beta * beta - alpha * alpha) / ((2 * kk + ab) * (2 * kk + ab + 2))
    a = np.zeros(n + 1)
    if n >= 1:
        a[1] = math.sqrt(4.0 * (1 + alpha) * (1 + beta) / ((2 + ab) ** 2 * (3 + ab)))
    if n >= 2:
        kk = k[2:]
        num = 4.0 * kk * (kk + alpha) * (kk + beta) * (kk + ab)
        den = (2 * kk + ab) ** 2 * (2 * kk + ab + 1) * (2 * kk + ab - 1)
        a[2:] = np.sqrt(num / den)
    return a, b


def _jacobi_p0(alpha, beta):
    ab = alpha + beta
    log_mu0 = ((ab + 1.0) * math.log(2.0) + math.lgamma(alpha + 1.0)
               + math.lgamma(beta + 1.0) - math.lgamma(ab + 2.0))
    return math.exp(-0.5 * log_mu0)


def jacobi_orthonormal(alpha, beta, x, m0, m1):
    """p_m(x_j) of the orthonormal Jacobi system, rows x, columns m0 .. m1-1 (m0 >= 0)."""
    x = np.asarray(x, dtype=np.float64)
    a, b = jacobi_coefficients(max(m1, 1), alpha, beta)
    out = np.empty((x.size, m1 - m0))
    p_prev = np.zeros_like(x)
    p = np.full_like(x, _jacobi_p0(alpha, beta))
    for m in range(m1):
        if m >= m0:
            out[:, m - m0] = p
        if m + 1 < m1:
            p_next = ((x - b[m]) * p - a[m] * p_prev) / a[m + 1]
            p_prev, p = p, p_next
    return out


def jacobi_pn_dpn(N, alpha, beta, x):
    """(p_N(x), p_N'(x)) of the orthonormal system, for Newton on the nodes."""
    a, b = jacobi_coefficients(N, alpha, beta)
    p_prev = np.zeros_like(x)
    p = np.full_like(x, _jacobi_p0(alpha, beta))
    d_prev = np.zeros_like(x)
    d = np.zeros_like(x)
    for m in range(N):
        p_next = ((x - b[m]) * p - a[m] * p_prev) / a[m + 1]
        d_next = ((x - b[m]) * d + p - a[m] * d_prev) / a[m + 1]
        p_prev, p, d_prev, d = p, p_next, d, d_next
    return p, d


# --------------------------------------------------------------------------- Laguerre

def laguerre_fn(x, m0, m1):
    """l_m(x_j) = exp(-x_j/2) L_m(x_j), rows x, columns m0 .. m1-1 (m0 >= 0)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((x.size, m1 - m0))
    mant, E = exp_neg_scaled(0.5 * x)
    l_prev = np.zeros_like(x)
    l = mant
    for m in range(m1):
        if m >= m0:
            out[:, m - m0] = np.ldexp(l, E)
        if m + 1 < m1:
            l_next = ((2 * m + 1 - x) * l - m * l_prev) / (m + 1)
            l_prev, l = l, l_next
            big = np.abs(l) > _BIG
            if np.any(big):
                l[big] *= _RESCALE
                l_prev[big] *= _RESCALE
                E[big] += 500
    return out


def laguerre_ln_dln(N, x):
    """(L_N(x), L_N'(x)) up to a common positive factor, for Newton on the nodes."""
    L_prev = np.zeros_like(x)
    L = np.ones_like(x)
    d_prev = np.zeros_like(x)
    d = np.zeros_like(x)
    for m in range(N):
        L_next = ((2 * m + 1 - x) * L - m * L_prev) / (m + 1)
        d_next = ((2 * m + 1 - x) * d - L - m * d_prev) / (m + 1)
        L_prev, L, d_prev, d = L, L_next, d, d_next
        big = np.maximum(np.abs(L), np.abs(d)) > _BIG
        if np.any(big):
            for arr in (L_prev, L, d_prev, d):
                arr[big] *= _RESCALE
    return L, d


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _two_prod(a, b):
    p = a * b
    ca, cb = 134217729.0 * a, 134217729.0 * b   # Veltkamp splitting, 2^27 + 1
    ah = ca - (ca - a)
    al = a - ah
    bh = cb - (cb - b)
    bl = b - bh
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


def _dd_norm(hi, lo):
    s = hi + lo
    return s, lo - (s - hi)


def _dd_mul(ah, al, bh, bl):
    p, e = _two_prod(ah, bh)
    return _dd_norm(p, e + (ah * bl + al * bh))


def _dd_sub(ah, al, bh, bl):
    s, e = _two_sum(ah, -bh)
    return _dd_norm(s, e + (al - bl))


def _dd_div_int(ah, al, d):
    q = ah / d
    p, e = _two_prod(q, d)
    return _dd_norm(q, ((ah - p) - e + al) / d)


def laguerre_ln_dln_dd(N, x):
    """(L_N(x), L_N'(x)) by the recurrence in double-double arithmetic, up to a
    common positive factor.  Near x = 0 the recurrence has a double
    characteristic root and float64 rounding grows like k^2 eps, which leaves
    the smallest roots with ~1e-11 relative error; the double-double pass is
    used for one final Newton correction."""
    x = np.asarray(x, dtype=np.float64)
    z = np.zeros_like(x)
    L_prev = (z.copy(), z.copy())
    L = (np.ones_like(x), z.copy())
    d_prev = (z.copy(), z.copy())
    d = (z.copy(), z.copy())
    for m in range(N):
        c = _two_sum(np.full_like(x, 2.0 * m + 1.0), -x)          # 2m+1-x, exact
        t = _dd_mul(c[0], c[1], L[0], L[1])
        mL = _dd_mul(np.full_like(x, float(m)), z, L_prev[0], L_prev[1])
        t = _dd_sub(t[0], t[1], mL[0], mL[1])
        L_next = _dd_div_int(t[0], t[1], m + 1.0)
        u = _dd_mul(c[0], c[1], d[0], d[1])
        u = _dd_sub(u[0], u[1], L[0], L[1])
        md = _dd_mul(np.full_like(x, float(m)), z, d_prev[0], d_prev[1])
        u = _dd_sub(u[0], u[1], md[0], md[1])
        d_next = _dd_div_int(u[0], u[1], m + 1.0)
        L_prev, L, d_prev, d = L, L_next, d, d_next
        big = np.maximum(np.abs(L[0]), np.abs(d[0])) > _BIG
        if np.any(big):
            for pair in (L_prev, L, d_prev, d):
                pair[0][big] *= _RESCALE
                pair[1][big] *= _RESCALE
    return L[0] + L[1], d[0] + d[1]


# --------------------------------------------------------------------------- Hermite

def hermite_fn(x, m0, m1):
    """psi_m(x_j) = exp(-x_j^2/2) h_m(x_j), rows x, columns m0 .. m1-1 (m0 >= 0)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((x.size, m1 - m0))
    hi, lo = exact_square(x)
    mant, E = exp_neg_scaled(0.5 * hi)
    mant = mant * (1.0 - 0.5 * lo) * math.pi ** -0.25
    p_prev = np.zeros_like(x)
    p = mant
    for m in range(m1):
        if m >= m0:
            out[:, m - m0] = np.ldexp(p, E)
        if m + 1 < m1:
            p_next = math.sqrt(2.0 / (m + 1)) * x * p - math.sqrt(m / (m + 1.0)) * p_prev
            p_prev, p = p, p_next
            big = np.abs(p) > _BIG
            if np.any(big):
                p[big] *= _RESCALE
                p_prev[big] *= _RESCALE
                E[big] += 500
    return out


def hermite_hn_dhn(N, x):
    """(h_N(x), h_N'(x)) up to a common positive factor, for Newton on the nodes."""
    h_prev = np.zeros_like(x)
    h = np.ones_like(x)
    d_prev = np.zeros_like(x)
    d = np.zeros_like(x)
    for m in range(N):
        c1 = math.sqrt(2.0 / (m + 1))
        c0 = math.sqrt(m / (m + 1.0))
        h_next = c1 * x * h - c0 * h_prev
        d_next = c1 * (h + x * d) - c0 * d_prev
        h_prev, h, d_prev, d = h, h_next, d, d_next
        big = np.maximum(np.abs(h), np.abs(d)) > _BIG
        if np.any(big):
            for arr in (h_prev, h, d_prev, d):
                arr[big] *= _RESCALE
    return h, d
