"""Coefficients of the polynomial that the FP64 exponential in csrc/equilibrium.h
evaluates after Cody and Waite's argument reduction: the degree-10 polynomial
of least maximum relative error for e^r on |r| <= ln(2)/2, found with the
Remez exchange algorithm in 60-digit arithmetic (mpmath).

    python -m paper_1910_13515_amd.exp_minimax

prints the levelled error and the coefficients c_0..c_10 (p(r) = sum c_j r^j)
as decimal and C hexadecimal literals.  Not used at run time.
"""
from __future__ import annotations


def remez(degree: int = 10, digits: int = 60, grid: int = 4000, iterations: int = 30):
    import mpmath as mp

    mp.mp.dps = digits
    a = mp.log(2) / 2
    n = degree
    # reference points: the extrema of the Chebyshev polynomial of degree n + 1
    pts = [a * mp.cos(mp.pi * k / (n + 1)) for k in range(n + 2)][::-1]
    xs = [-a + 2 * a * k / grid for k in range(grid + 1)]
    coef, level, worst = None, None, None
    for it in range(iterations):
        # p(x_i) - e^{x_i} = (-1)^i E e^{x_i}: the relative error levelled at the reference
        A = mp.matrix(n + 2, n + 2)
        b = mp.matrix(n + 2, 1)
        for i, x in enumerate(pts):
            for j in range(n + 1):
                A[i, j] = x ** j
            A[i, n + 1] = (-1) ** i * mp.exp(x)
            b[i] = mp.exp(x)
        sol = mp.lu_solve(A, b)
        coef = [sol[j] for j in range(n + 1)]
        level = abs(sol[n + 1])
        err = [(mp.polyval(coef[::-1], x) - mp.exp(x)) / mp.exp(x) for x in xs]
        worst = max(abs(e) for e in err)
        # new reference: the largest error between consecutive sign changes
        runs, start = [], 0
        for k in range(1, grid + 1):
            if mp.sign(err[k]) != mp.sign(err[k - 1]):
                runs.append((start, k - 1))
                start = k
        runs.append((start, grid))
        if len(runs) != n + 2:
            raise RuntimeError(f"{len(runs)} alternations, expected {n + 2}")
        pts = [xs[max(range(s0, s1 + 1), key=lambda k: abs(err[k]))] for s0, s1 in runs]
        if it > 3 and abs(worst - level) / worst < 1e-6:
            break
    return coef, level, worst


def main():
    import mpmath as mp

    coef, level, worst = remez()
    print(f"levelled relative error {mp.nstr(level, 6)}, largest on the grid {mp.nstr(worst, 6)}")
    for j, c in enumerate(coef):
        print(j, mp.nstr(c, 25), float(c).hex())


if __name__ == "__main__":
    main()
