// Device arithmetic of the 13-moment exponential equilibrium (Sec. 2 of the
// paper, Eq. eq:discrete-equilibrium) and its Newton-Raphson solve (Sec. 3 and
// the algorithm table of Sec. 5), templated on the arithmetic type C (double
// or float).  Everything is written per lane (one cell per lane) with all
// loops unrolled at compile time so that the lattice constants fold into the
// instruction stream.
#pragma once

#include "d3q39.h"
#include "slot.h"

namespace lbm13 {

template <class C>
__device__ __forceinline__ C dexp(C x);
template <>
__device__ __forceinline__ double dexp<double>(double x) { return exp(x); }
template <>
__device__ __forceinline__ float dexp<float>(float x) { return expf(x); }

template <class C>
__device__ __forceinline__ C dlog(C x);
template <>
__device__ __forceinline__ double dlog<double>(double x) { return log(x); }
template <>
__device__ __forceinline__ float dlog<float>(float x) { return logf(x); }

template <class C>
__device__ __forceinline__ C dsqrt(C x);
template <>
__device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }
template <>
__device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }

// Maxwell-Boltzmann targets per unit density (Eq. eq:EqMomentsTensor, the 13
// constraints of Eq. eq:13constraints; the contracted third moment is
// u_a (|u|^2 + (D + 2) T) with D = 3).
template <class C>
__device__ __forceinline__ void mb_targets(const C u[3], C T, C m[kM])
{
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const C h = uu + C(5) * T;
    m[0] = C(1);
    m[1] = u[0];
    m[2] = u[1];
    m[3] = u[2];
    m[4] = u[0] * u[0] + T;
    m[5] = u[1] * u[1] + T;
    m[6] = u[2] * u[2] + T;
    m[7] = u[0] * u[1];
    m[8] = u[0] * u[2];
    m[9] = u[1] * u[2];
    m[10] = h * u[0];
    m[11] = h * u[1];
    m[12] = h * u[2];
}

// exp(phi_i . lam) for the rest velocity (f0) and both members of every pair
template <int P, class C>
__device__ __forceinline__ void eval_pair(const C *lam, C *fp, C *fm)
{
    const C e = exponent_part<false, P>(lam, BasisSeq{});
    const C o = exponent_part<true, P>(lam, BasisSeq{});
    fp[P] = dexp(e + o);
    fm[P] = dexp(e - o);
}

template <class C, int... P>
__device__ __forceinline__ void eval_pairs(const C *lam, C *fp, C *fm, std::integer_sequence<int, P...>)
{
    (eval_pair<P>(lam, fp, fm), ...);
}

template <class C>
__device__ __forceinline__ void eval_exponentials(const C lam[kM], C &f0, C fp[kPairs], C fm[kPairs])
{
    f0 = dexp(lam[0]);
    eval_pairs(lam, fp, fm, PairSeq{});
}

// G_k = sum_i exp(phi_i . lam) phi_ik - m_k from pair sums s and differences a
template <class C, int... K>
__device__ __forceinline__ void residual_impl(C f0, const C *s, const C *a, const C *m, C *G,
                                              std::integer_sequence<int, K...>)
{
    ((G[K] = ((K == 0) ? f0 : C(-0.0)) + basis_sum<K>(basis_odd(K) ? a : s, PairSeq{}) - m[K]), ...);
}

template <int K, int L, class C>
__device__ __forceinline__ C jac_entry(C f0, const C *s, const C *a)
{
    constexpr bool odd = basis_odd(K) != basis_odd(L);
    C v = gram_sum<K, L>(odd ? a : s, PairSeq{});
    if constexpr (K == 0 && L == 0) v = f0 + v;
    return v;
}

template <int L, class C, int... K>
__device__ __forceinline__ void jac_row(C f0, const C *s, const C *a, C (&J)[kM][kM], std::integer_sequence<int, K...>)
{
    ((J[L][K] = jac_entry<K, L>(f0, s, a)), ...);
}

// lower triangle of J_kl = sum_i exp(phi_i . lam) phi_ik phi_il
template <class C, int... L>
__device__ __forceinline__ void jacobian_impl(C f0, const C *s, const C *a, C (&J)[kM][kM],
                                              std::integer_sequence<int, L...>)
{
    (jac_row<L>(f0, s, a, J, std::make_integer_sequence<int, L + 1>{}), ...);
}

// Solve J d = G.  The paper inverts J; J is symmetric positive definite, so
// a Cholesky factorisation gives the same d.  Returns false if a pivot is not
// positive (or not a number).
template <class C>
__device__ __forceinline__ bool cholesky_solve(C (&J)[kM][kM], const C G[kM], C d[kM])
{
    bool ok = true;
    C rdiag[kM];
#pragma unroll
    for (int j = 0; j < kM; ++j) {
        C s = J[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= J[j][k] * J[j][k];
        ok = ok && (s > C(0));
        const C r = C(1) / dsqrt(s);
        rdiag[j] = r;
#pragma unroll
        for (int i = j + 1; i < kM; ++i) {
            C t = J[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= J[i][k] * J[j][k];
            J[i][j] = t * r;
        }
    }
    C y[kM];
#pragma unroll
    for (int i = 0; i < kM; ++i) {
        C t = G[i];
#pragma unroll
        for (int k = 0; k < i; ++k) t -= J[i][k] * y[k];
        y[i] = t * rdiag[i];
    }
#pragma unroll
    for (int i = kM - 1; i >= 0; --i) {
        C t = y[i];
#pragma unroll
        for (int k = i + 1; k < kM; ++k) t -= J[k][i] * d[k];
        d[i] = t * rdiag[i];
    }
    return ok;
}

// Multipliers of the Maxwellian shape (cold start): lam_1 = u/T,
// lam_2 = -delta/(2T), lam_3 = 0, lam_0 normalising sum_i exp(...) to 1.
template <class C>
__device__ __forceinline__ void cold_guess(const C u[3], C T, C lam[kM])
{
#pragma unroll
    for (int k = 0; k < kM; ++k) lam[k] = C(0);
    lam[1] = u[0] / T;
    lam[2] = u[1] / T;
    lam[3] = u[2] / T;
    lam[4] = lam[5] = lam[6] = C(-0.5) / T;
    C f0, fp[kPairs], fm[kPairs];
    eval_exponentials(lam, f0, fp, fm);
    C s = f0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) s += fp[p] + fm[p];
    lam[0] = -dlog(s);
}

// Newton-Raphson for the multipliers, warm-started from lam.  Stopping rule:
// max_k |G_k| <= tol * max(1, max_k |m_k|).  Step halving while the Euclidean
// norm of G does not decrease (at most 39 halvings, then the step is taken).
// If the warm start fails (cap reached, J not positive definite, or a value
// not finite) the solve restarts once from the Maxwellian shape with cap
// maxit_cold.  On return lam, f0, fp, fm hold the last accepted iterate and
// iters the number of accepted updates of the final attempt (maxit if both
// attempts failed).
template <class C>
__device__ __forceinline__ int solve_multipliers(const C m[kM], const C u[3], C T, C lam[kM], C &f0, C fp[kPairs],
                                                 C fm[kPairs], C tol, int maxit, int maxit_cold, int &iters)
{
    C scale = C(1);
#pragma unroll
    for (int k = 0; k < kM; ++k) scale = fabs(m[k]) > scale ? fabs(m[k]) : scale;
    const C bound = tol * scale;

    C base[kM], d[kM];
#pragma unroll
    for (int k = 0; k < kM; ++k) {
        base[k] = lam[k];
        d[k] = C(0);
    }
    C t = C(0);
    C n0 = C(0);
    int it = 0, ls = 0, cap = maxit;
    bool fresh = true, cold = false;
    int status = kFailed;
    for (;;) {
#pragma unroll
        for (int k = 0; k < kM; ++k) lam[k] = base[k] - t * d[k];
        eval_exponentials(lam, f0, fp, fm);
        C s[kPairs], a[kPairs];
#pragma unroll
        for (int p = 0; p < kPairs; ++p) {
            s[p] = fp[p] + fm[p];
            a[p] = fp[p] - fm[p];
        }
        C G[kM];
        residual_impl(f0, s, a, m, G, BasisSeq{});
        C n2 = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) n2 += G[k] * G[k];
        n2 = dsqrt(n2);
        if (!fresh && !(n2 < n0) && ls < 39) {
            t *= C(0.5);
            ++ls;
            continue;
        }
        if (!fresh) ++it;
        fresh = false;
        C r = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const C g = fabs(G[k]);
            r = (g <= r) ? r : g;  // NaN propagates
        }
        if (r <= bound) {
            status = cold ? kConvergedCold : kConverged;
            break;
        }
        bool bad = !(r - r == C(0)) || it >= cap;  // not finite, or cap reached
        if (!bad) {
            C J[kM][kM];
            jacobian_impl(f0, s, a, J, BasisSeq{});
            bad = !cholesky_solve(J, G, d);
        }
        if (bad) {
            if (cold) {
                status = kFailed;
                break;
            }
            cold = true;
            cold_guess(u, T, base);
#pragma unroll
            for (int k = 0; k < kM; ++k) d[k] = C(0);
            t = C(0);
            it = 0;
            ls = 0;
            cap = maxit_cold;
            fresh = true;
            continue;
        }
#pragma unroll
        for (int k = 0; k < kM; ++k) base[k] = lam[k];
        t = C(1);
        ls = 0;
        n0 = n2;
    }
    iters = status == kFailed ? maxit : it;
    return status;
}

// equilibrium per unit density of velocity i from the solve's exponentials
template <int I, class C>
__device__ __forceinline__ C feq_of(C f0, const C *fp, const C *fm)
{
    if constexpr (I == 0) return f0;
    else if constexpr (((I - 1) & 1) == 0) return fp[(I - 1) >> 1];
    else return fm[(I - 1) >> 1];
}

}  // namespace lbm13
