"""Generator of the polynomial coefficients of the device sin/cos and arctangent
(ah_device.hpp).

sincos (double): the device reduces x by multiples of pi, x = k*pi + r with
|r| <= pi/2, and evaluates
    sin r = r + r^3 * P(r^2),    cos r = 1 + r^2 * Q(r^2),
flipping both signs for odd k.  P is the minimax fit (relative error of sin r)
and Q the minimax fit (absolute error of cos r) on 0 <= r <= pi/2.  The float
sin/cos reduces by multiples of 2 pi and ends in the hardware sine and cosine;
only its reduction constants are printed here.

arctangent (FP32 phase of the winding filter): atan a = a + a^3 * T(a^2) on
0 <= a <= 1 (the ratio of the smaller to the larger of |x|, |y|), minimax in
relative error.

All fits use the Remez exchange algorithm on a dense grid in 50-digit
arithmetic (mpmath), then round to the working precision.  Run with no
arguments to print every set; the header holds the printed values.
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 50
HALF_PI = mp.pi / 2


def remez(n, target, weight, grid_pts=4000, iters=40, U=HALF_PI ** 2):
    """Minimax polynomial sum_j c_j u^j (n terms) of target(u) on (0, U] for the
    weighted error weight(u) * (p(u) - target(u))."""
    grid = [U * (1 - mp.cos(mp.pi * (i + 0.5) / grid_pts)) / 2 for i in range(grid_pts)]
    grid[-1] = U
    tv = [target(u) for u in grid]
    wv = [weight(u) for u in grid]
    ref = [int(round((grid_pts - 1) * (1 - mp.cos(mp.pi * i / n)) / 2)) for i in range(n + 1)]
    ref = sorted(set(max(1, i) for i in ref))
    c, E = None, None
    for _ in range(iters):
        A = mp.matrix(n + 1, n + 1)
        b = mp.matrix(n + 1, 1)
        for row, gi in enumerate(ref):
            u = grid[gi]
            for j in range(n):
                A[row, j] = u ** j
            A[row, n] = (-1) ** row / wv[gi]
            b[row] = tv[gi]
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(n)]
        E = abs(sol[n])
        err = [wv[i] * (mp.polyval(c[::-1], grid[i]) - tv[i]) for i in range(grid_pts)]
        # new reference: the extremum of each run of equal error sign
        runs, cur = [], None
        for i, e in enumerate(err):
            s = e >= 0
            if cur is None or s != cur[0]:
                cur = [s, i]
                runs.append(cur)
            elif abs(e) > abs(err[cur[1]]):
                cur[1] = i
        idx = [r[1] for r in runs]
        while len(idx) > n + 1:   # drop the smaller end
            if abs(err[idx[0]]) < abs(err[idx[-1]]):
                idx.pop(0)
            else:
                idx.pop()
        if len(idx) < n + 1:
            break
        new_max = max(abs(e) for e in err)
        ref = idx
        if new_max - E < mp.mpf(10) ** -6 * E:
            break
    return c, max(abs(wv[i] * (mp.polyval(c[::-1], grid[i]) - tv[i])) for i in range(grid_pts))


def sin_tail(u):
    r = mp.sqrt(u)
    return (mp.sin(r) - r) / (r * u) if u > 0 else mp.mpf(-1) / 6


def cos_tail(u):
    return (mp.cos(mp.sqrt(u)) - 1) / u if u > 0 else mp.mpf(-1) / 2


def atan_tail(u):
    a = mp.sqrt(u)
    return (mp.atan(a) - a) / (a * u) if u > 0 else mp.mpf(-1) / 3


def fit_atan(n):
    return remez(n, atan_tail, lambda u: u * mp.sqrt(u) / mp.atan(mp.sqrt(u)), U=mp.mpf(1))


def fit(n_sin, n_cos):
    ps, es = remez(n_sin, sin_tail, lambda u: u * mp.sqrt(u) / mp.sin(mp.sqrt(u)))
    pc, ec = remez(n_cos, cos_tail, lambda u: u)
    return ps, es, pc, ec


def rounded(v, name):
    """Shortest decimal that reads back as v rounded to the working precision."""
    if name == "float":
        return np.format_float_scientific(np.float32(float(v)), unique=True) + "f"
    return repr(float(v))


def main():
    ps, es, pc, ec = fit(8, 8)
    print(f"// double: sin rel. error {mp.nstr(es, 3)}, cos abs. error {mp.nstr(ec, 3)}")
    print("P (r^0 first):", ", ".join(rounded(v, "double") for v in ps))
    print("Q (r^0 first):", ", ".join(rounded(v, "double") for v in pc))
    lo = mp.pi - mp.mpf(float(mp.pi))
    print("1/pi, pi high, pi low:", rounded(1 / mp.pi, "double"), rounded(mp.pi, "double"),
          rounded(lo, "double"))
    hi = mp.mpf(float(np.float32(float(2 * mp.pi))))
    print("// float: 1/(2 pi), 2 pi high, 2 pi low:", rounded(1 / (2 * mp.pi), "float"),
          rounded(hi, "float"), rounded(2 * mp.pi - hi, "float"))

    pa, ea = fit_atan(7)
    print(f"// float arctangent: rel. error {mp.nstr(ea, 3)}")
    print("T (a^0 first):", ", ".join(rounded(v, "float") for v in pa))
    print("pi/2, pi:", rounded(HALF_PI, "float"), rounded(mp.pi, "float"))


if __name__ == "__main__":
    main()
