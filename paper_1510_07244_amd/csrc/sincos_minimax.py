"""Coefficients of the sine and cosine polynomials of bem_device.h.

After the Cody-Waite reduction x = k pi + r to r in [-pi/2, pi/2],
t = r^2 in [0, T], T = (pi/2)^2:

    sin r ~ r + r^3 P(t),   cos r ~ 1 - t/2 + t^2 Q(t)

(sin x and cos x are then those of r, both negated for odd k).  P is
chosen to minimise the largest error relative to sin r (weight
t^(3/2) / sin(sqrt t)), Q the largest absolute error of cos r (weight t^2:
cos r vanishes at the interval's ends, where only absolute accuracy makes
sense -- it is what the kernel e^{i kappa r} needs).  FP64: P of degree 7,
Q of degree 6; FP32: degree 3 each.  Method: the Remez exchange algorithm
(E. Ya. Remez, 1934) in x86 long double, applied to the part of the Taylor
series beyond the polynomial's degree -- the polynomial is the Taylor
polynomial plus a minimax correction, so the levelled linear systems solve
for quantities of the size of the error, not of the coefficients -- on t in
[1e-3 T, T] (below, the weights make every error negligible).  Run as a
script to print the coefficients as hexadecimal floats;
tests/test_host_sincos.py checks the header's against this construction's
error bounds.
"""
import numpy as np

L = np.longdouble
T = L(np.pi / 2) ** 2


def _fact(n):
    r = L(1)
    for k in range(2, n + 1):
        r *= k
    return r


def _series(t, first, step_den, count, shift):
    """sum_{n >= first} (-1)^n t^(n - shift) / (step_den * n + ...)! helper:
    terms (-1)^n t^(n - shift) / (2n + step_den)!"""
    t = np.asarray(t, dtype=L)
    s = np.zeros_like(t)
    p = t ** (first - shift)
    for n in range(first, first + count):
        s += (-1) ** n * p / _fact(2 * n + step_den)
        p = p * t
    return s


def sin_f(t):
    """(sin r - r) / r^3 as a function of t = r^2."""
    return _series(t, 1, 1, 24, 1)


def cos_f(t):
    """(cos r - 1 + r^2 / 2) / r^4 as a function of t = r^2."""
    return _series(t, 2, 0, 24, 2)


def sin_w(t):
    t = np.asarray(t, dtype=L)
    r = np.sqrt(t)
    return t * r / (r * (1 + t * sin_f(t)))


def cos_w(t):
    """Absolute error of cos r."""
    t = np.asarray(t, dtype=L)
    return t * t


def _solve(A, b):
    """Gaussian elimination with partial pivoting in long double."""
    A = [list(r) for r in A]
    b = list(b)
    n = len(b)
    for i in range(n):
        p = max(range(i, n), key=lambda r: abs(A[r][i]))
        A[i], A[p], b[i], b[p] = A[p], A[i], b[p], b[i]
        for r in range(i + 1, n):
            m = A[r][i] / A[i][i]
            for c in range(i, n):
                A[r][c] -= m * A[i][c]
            b[r] -= m * b[i]
    x = [L(0)] * n
    for i in range(n - 1, -1, -1):
        x[i] = (b[i] - sum(A[i][c] * x[c] for c in range(i + 1, n))) / A[i][i]
    return x


def _remez(fun, weight, a, b, deg, iters=25, npts=20001):
    """Minimax polynomial of degree `deg` to fun in the weight on [a, b]."""
    n = deg + 2
    k = np.arange(n)
    ref = ((a + b) / 2 - (b - a) / 2 * np.cos(np.pi * k / (n - 1))).astype(L)
    grid = np.linspace(float(a), float(b), npts).astype(L)
    fg, wg = fun(grid), weight(grid)
    c, E = None, None
    for _ in range(iters):
        wr = weight(ref)
        A = [[ref[i] ** j for j in range(deg + 1)] + [L((-1) ** i) / wr[i]] for i in range(n)]
        sol = _solve(A, fun(ref))
        c, E = sol[:-1], sol[-1]
        P = np.zeros_like(grid)
        for cj in c[::-1]:
            P = P * grid + cj
        err = (P - fg) * wg
        sgn = np.where(err >= 0, 1, -1)
        ext, st = [], 0
        for i in range(1, grid.size):
            if sgn[i] != sgn[i - 1]:
                ext.append(st + int(np.argmax(np.abs(err[st:i]))))
                st = i
        ext.append(st + int(np.argmax(np.abs(err[st:]))))
        while len(ext) > n:  # drop the smaller end (keeps the alternation)
            ext.pop(0 if abs(err[ext[0]]) < abs(err[ext[-1]]) else -1)
        if len(ext) < n:
            break
        ref = grid[ext]
    return c, abs(float(E))


def coefficients(kind, deg):
    """Long-double coefficients (lowest first) of P (kind 'sin') or Q
    ('cos') of degree deg, and the levelled weighted error."""
    if kind == "sin":
        taylor = [L((-1) ** n) / _fact(2 * n + 1) for n in range(1, deg + 2)]
        tail = lambda t: _series(t, deg + 2, 1, 24, 1)
        w = sin_w
    else:
        taylor = [L((-1) ** n) / _fact(2 * n) for n in range(2, deg + 3)]
        tail = lambda t: _series(t, deg + 3, 0, 24, 2)
        w = cos_w
    d, E = _remez(tail, w, T * L(1e-3), T, deg)
    return [a + b for a, b in zip(taylor, d)], E


def max_rel_error(kind, coefs, npts=200001):
    """Largest error over t in [0, T] of the polynomial with the given
    (rounded) coefficients, in long double: relative to sin r for the sine,
    absolute for the cosine."""
    t = np.linspace(0.0, float(T), npts).astype(L)
    P = np.zeros_like(t)
    for c in coefs[::-1]:
        P = P * t + L(c)
    if kind == "sin":
        return float(np.max(np.abs((P - sin_f(t)) * sin_w(np.maximum(t, L(1e-300))))))
    return float(np.max(np.abs((P - cos_f(t)) * cos_w(t))))


if __name__ == "__main__":
    for kind, deg, typ in (("sin", 7, np.float64), ("cos", 6, np.float64),
                           ("sin", 3, np.float32), ("cos", 3, np.float32)):
        c, E = coefficients(kind, deg)
        r = [typ(x) for x in c]
        print(kind, typ.__name__, "levelled", E, "rounded", max_rel_error(kind, r))
        print("   ", [float(x).hex() for x in r])
