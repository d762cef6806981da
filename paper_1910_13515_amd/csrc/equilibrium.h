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
__device__ __forceinline__ float dexp<float>(float x) { return __expf(x); }  // v_exp_f32 on x log2(e)

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

// 1/sqrt(x) and 1/x: exact division in FP64; the hardware approximations
// (about 1 ulp) in the FP32 path.
// FP64: the hardware estimates refined by two Newton steps each (each step
// squares the relative error), in place of the full-precision division and
// square-root sequences; used for the Cholesky pivots and the sensor, whose
// results need accuracy to a few ulp, not correct rounding
__device__ __forceinline__ double rsqrt_(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-(x * y), y, 1.0);  // 1 - x y^2
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-(x * y), y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);  // 1 - x y
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

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

// Target k of mb_targets evaluated from (u, T, h = |u|^2 + 5T)
template <int K, class C>
__device__ __forceinline__ C target(const C u[3], C T, C h)
{
    if constexpr (K == 0) return C(1);
    else if constexpr (K <= 3) return u[K - 1];
    else if constexpr (K <= 6) return u[K - 4] * u[K - 4] + T;
    else if constexpr (K == 7) return u[0] * u[1];
    else if constexpr (K == 8) return u[0] * u[2];
    else if constexpr (K == 9) return u[1] * u[2];
    else return h * u[K - 10];
}

// G_k = sum_i exp(phi_i . lam) phi_ik - m_k from pair sums s and differences a
template <class C, int... K>
__device__ __forceinline__ void residual_impl(C f0, const C *s, const C *a, const C u[3], C T, C h, C *G,
                                              std::integer_sequence<int, K...>)
{
    ((G[K] = ((K == 0) ? f0 : C(-0.0)) + basis_sum<K>(basis_odd(K) ? a : s, PairSeq{}) - target<K>(u, T, h)), ...);
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
        const C r = rsqrt_(s);
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
// attempts failed).  The targets m are evaluated from (u, T) where needed.
template <class C>
__device__ __forceinline__ int solve_multipliers(const C u[3], C T, C lam[kM], C &f0, C fp[kPairs], C fm[kPairs],
                                                 C tol, int maxit, int maxit_cold, int &iters, C (&resid)[5])
{
    C m[kM];
    mb_targets(u, T, m);
    C scale = C(1);
#pragma unroll
    for (int k = 0; k < kM; ++k) scale = fabs(m[k]) > scale ? fabs(m[k]) : scale;
    const C bound = tol * scale;
    const C h = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + C(5) * T;

    // lam holds the trial point lam_acc - t d; a rejected trial moves back by
    // half its step (t -> t/2)
    C d[kM];
#pragma unroll
    for (int k = 0; k < kM; ++k) d[k] = C(0);
    C t = C(0);
    C n0 = C(0);
    int it = 0, ls = 0, cap = maxit;
    bool fresh = true, cold = false, floor_stop = false;
    bool near = false;  // the last accepted iterate is within 8 times the bound
    int status = kFailed;
    for (;;) {
        eval_exponentials(lam, f0, fp, fm);
        C s[kPairs], a[kPairs];
#pragma unroll
        for (int p = 0; p < kPairs; ++p) {
            s[p] = fp[p] + fm[p];
            a[p] = fp[p] - fm[p];
        }
        C G[kM];
        residual_impl(f0, s, a, u, T, h, G, BasisSeq{});
        C n2 = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) n2 += G[k] * G[k];
        n2 = dsqrt(n2);
        C r = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const C g = fabs(G[k]);
            r = (g <= r) ? r : g;  // NaN propagates
        }
        // the full step does not lower the residual, but the accepted iterate
        // and the step's end are both within 8 times the bound: the residual
        // sits at the round-off floor; the step is taken and the solve stops
        floor_stop = !fresh && !(n2 < n0) && ls == 0 && near && r <= C(8) * bound;
        if (!fresh && !(n2 < n0) && ls < 39 && !floor_stop) {
            t *= C(0.5);
            ++ls;
#pragma unroll
            for (int k = 0; k < kM; ++k) lam[k] += t * d[k];
            continue;
        }
        if (!fresh) ++it;
        fresh = false;
        // residuals of the collision invariants at the accepted iterate:
        // mass, momentum, and sum_i f_i |xi_i|^2 (trace of the second moment)
        resid[0] = G[0];
        resid[1] = G[1];
        resid[2] = G[2];
        resid[3] = G[3];
        resid[4] = G[4] + G[5] + G[6];
        near = r <= C(8) * bound;
        if (r <= bound || floor_stop) {
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
            cold_guess(u, T, lam);
            it = 0;
            ls = 0;
            cap = maxit_cold;
            fresh = true;
            continue;
        }
        t = C(1);
        ls = 0;
        n0 = n2;
#pragma unroll
        for (int k = 0; k < kM; ++k) lam[k] -= d[k];
    }
    if (status == kFailed) {
        // no equilibrium: leave finite values behind (the caller does not
        // relax such a cell, and omega = 0 times a finite difference is 0);
        // zero residuals keep the invariant projection a no-op
        f0 = C(0);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) fp[p] = fm[p] = C(0);
#pragma unroll
        for (int k = 0; k < 5; ++k) resid[k] = C(0);
    }
    iters = status == kFailed ? maxit : it;
    return status;
}

// Remove the residual of the collision invariants from an equilibrium (per
// unit density) that satisfies the constraints only to a tolerance:
// f_i += w_i (a + b . xi_i + c |xi_i|^2) with the isotropic rest weights w
// of each shell, so that sum_i f_i (1, xi_i, |xi_i|^2) is exact.  With
// isotropic weights the five equations decouple: b_a = -R_a / W2 and (a, c)
// from the 2x2 system [[W0, Wq], [Wq, Wqq]] (a, c) = -(R_0, R_E), whose
// inverse is passed in (inv = {i00, i01, i11}).
template <int P, class C>
__device__ __forceinline__ void project_pair(C *fp, C *fm, C a, C c, const C b[3], const float *wshell)
{
    constexpr int cx = kPairVel[P][0], cy = kPairVel[P][1], cz = kPairVel[P][2];
    const C w = C(wshell[shell_of_q(pair_q(P))]);
    const C even = w * (a + C(pair_q(P)) * c);
    C odd = C(-0.0);
    odd = Term<cx>::add(odd, b[0]);
    odd = Term<cy>::add(odd, b[1]);
    odd = Term<cz>::add(odd, b[2]);
    odd *= w;
    fp[P] += even + odd;
    fm[P] += even - odd;
}

template <class C, int... P>
__device__ __forceinline__ void project_invariants(C &f0, C *fp, C *fm, const C (&resid)[5], const float *wshell,
                                                   const float *inv, float inv_w2, std::integer_sequence<int, P...>)
{
    const C a = -(C(inv[0]) * resid[0] + C(inv[1]) * resid[4]);
    const C c = -(C(inv[1]) * resid[0] + C(inv[2]) * resid[4]);
    const C b[3] = {-resid[1] * C(inv_w2), -resid[2] * C(inv_w2), -resid[3] * C(inv_w2)};
    f0 += C(wshell[0]) * a;
    (project_pair<P, C>(fp, fm, a, c, b, wshell), ...);
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
