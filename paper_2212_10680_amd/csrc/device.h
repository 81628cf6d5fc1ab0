// Device building blocks of the fugacity-based well-balanced LBM update on
// gfx950: lattice tables, the cubic-EOS log-fugacity, equilibrium, forcing and
// collision of one component at one node.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fl {

constexpr int kMaxComp = 4;

enum { kPR = 0, kSRK = 1, kVDW = 2 };

// Per-launch constants (passed by value as a kernel argument).
struct KParams {
    int nx, ny, nz;
    int N;                      // nx*ny*nz
    int eos;
    int force_level;            // 0: previous step's force in u; 1: this step's
    int standard;               // 1: standard-LBM form (eqForceGen), FP64 populations only
    int iso;                    // 1: isotropic lattice stencils in steps 6-7
    double RT, lnRT;
    double omega;               // 1/tau
    double cF;                  // 1 - 1/(2 tau)
    double s_j, s_nu, s_e, s_g; // MRT rates
    // (s_k - s_g) / |row k of the moment basis|^2 per group moment, set on the
    // host for the lattice: D3Q19 jx, jy, jz, then the five stress moments,
    // then the energy; D2Q9 jx, jy, the two stress moments, the energy
    double mrt_f[9];
    double b[kMaxComp];
    double M[kMaxComp];
    double aa[kMaxComp * kMaxComp];   // (a alpha)_ij
    double kap[kMaxComp * kMaxComp];  // kappa_ij = sqrt(kappa_i kappa_j)
    double sk[kMaxComp];              // sqrt(kappa_i)
};

// ---------------------------------------------------------------- lattices
// Directions are stored opposite pairs next to each other after the rest one.
template <int LAT>
struct Lat;

template <>
struct Lat<0> {  // D2Q9
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

template <>
struct Lat<1> {  // D3Q19
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

// ------------------------------------------------------------------- EOS
// Steps 3-5 at one node from the molar densities rt[i] (App. C mixing rules,
// eqPREOS/eqSRKEOS/eqvdwEOS, and ln f_i of eqfugupdatePR/SRK/VDW).  The
// density-explicit ln f is evaluated in the algebraically identical form
//   ln f_i = ln(rho~_i RT) - log1p(-eta) + (b_i/b_m)(Z-1)
//            + C (b_i/b_m - 2 s_i/(a alpha)_m) L,   eta = b_m rho~,
// with L = log1p(2 sqrt2 eta / (1 + (1-sqrt2) eta)) for PR and log1p(eta) for
// SRK: ln((v-b_m)/RT) and the ratio of the last logarithm are rewritten around
// 1 so that dilute vapor keeps full FP64 precision.  Returns false outside the
// domain (rho~_i <= 0, eta >= 1, non-finite).
template <int NC>
__device__ __forceinline__ bool eos_lnf(const KParams& kp, const double (&rt)[NC],
                                        double (&lnf)[NC], double* p_out) {
    constexpr double kSqrt2 = 1.4142135623730951;
    double r = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        r += rt[i];
        ok = ok && (rt[i] > 0.0);
    }
    const double inv = 1.0 / r;
    double x[NC], s[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) x[i] = rt[i] * inv;
    double bm = 0.0, am = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) bm += x[i] * kp.b[i];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        double si = 0.0;
#pragma unroll
        for (int j = 0; j < NC; ++j) si += x[j] * kp.aa[i * NC + j];
        s[i] = si;
        am += x[i] * si;
    }
    const double eta = bm * r;
    ok = ok && (eta < 1.0) && (r < 1e300);
    const double RT = kp.RT;
    const double l1 = log1p(-eta);             // ln(1 - eta)
    double zm1, l2, coef, p;
    if (kp.eos == kPR) {
        const double den = 1.0 + 2.0 * eta - eta * eta;
        zm1 = eta / (1.0 - eta) - am * r / (RT * den);
        l2 = log1p(2.0 * kSqrt2 * eta / (1.0 + (1.0 - kSqrt2) * eta));
        coef = am / (2.0 * kSqrt2 * bm * RT);
        p = r * RT / (1.0 - eta) - am * r * r / den;
    } else if (kp.eos == kSRK) {
        const double den = 1.0 + eta;
        zm1 = eta / (1.0 - eta) - am * r / (RT * den);
        l2 = log1p(eta);
        coef = am / (bm * RT);
        p = r * RT / (1.0 - eta) - am * r * r / den;
    } else {
        zm1 = 0.0;
        l2 = 0.0;
        coef = 0.0;
        p = r * RT / (1.0 - eta) - am * r * r;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        double l = log(rt[i]) + kp.lnRT - l1;
        if (kp.eos == kVDW)
            l += kp.b[i] * r / (1.0 - eta) - 2.0 * s[i] * r / RT;
        else
            l += kp.b[i] / bm * zm1 + coef * (kp.b[i] / bm - 2.0 * s[i] / am) * l2;
        lnf[i] = l;
        ok = ok && (l == l);
    }
    if (p_out) *p_out = p;
    return ok;
}

// --------------------------------------------- equilibrium, forcing, collision
// Scalars of one component at one node, in the collision precision T.
template <typename T>
struct CompState {
    T rho;        // rho_i (mass density)
    T ux, uy, uz; // barycentric velocity (step 1)
    T Fx, Fy, Fz; // component force F_i (step 7)
    T Gx, Gy, Gz; // grad rho_i (eq1stder)
};

// Well-balanced equilibrium without its rest-population density term
// (eq. eqLBEMCb, rho_0 = rho_0,i = 0): w_a rho [3 e.u + 9/2 (e.u)^2 - 3/2 u.u].
// The rest population adds rho_i itself.
template <typename L, typename T, int A>
__device__ __forceinline__ T geq_shape(const CompState<T>& c, T uu) {
    constexpr T ex = L::ex[A], ey = L::ey[A], ez = L::ez[A];
    const T eu = ex * c.ux + ey * c.uy + ez * c.uz;
    return T(L::w[A]) * c.rho * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * uu);
}

// Forcing term of eq. eqLBEMCfinal3 with c_s^2 = 1/3:
// w_a [F.((e-u)/cs2 + (u.e) e/cs4) + grad rho.(-u + (u.e) e/cs2 + (e^2/cs2 - D) u / 2)].
template <typename L, typename T, int A>
__device__ __forceinline__ T forcing(const CompState<T>& c, T uF, T uG) {
    constexpr T ex = L::ex[A], ey = L::ey[A], ez = L::ez[A];
    constexpr T e2 = ex * ex + ey * ey + ez * ez;
    constexpr T half_term = T(-1) + T(0.5) * (T(3) * e2 - T(L::D));
    const T eu = ex * c.ux + ey * c.uy + ez * c.uz;
    const T eF = ex * c.Fx + ey * c.Fy + ez * c.Fz;
    const T eG = ex * c.Gx + ey * c.Gy + ez * c.Gz;
    return T(L::w[A]) * (T(3) * eF - T(3) * uF + T(9) * eu * eF + half_term * uG + T(3) * eu * eG);
}

template <int I, int N>
struct Unroll {
    template <typename F>
    __device__ __forceinline__ static void run(F&& f) {
        f(std::integral_constant<int, I>{});
        Unroll<I + 1, N>::run(f);
    }
};
template <int N>
struct Unroll<N, N> {
    template <typename F>
    __device__ __forceinline__ static void run(F&&) {}
};

// Collision of one component.  gv[a] holds the stored populations (for the
// FP32 form the rest slot holds g_0 minus the reference density, and
// moving_sum is sum_{a != 0} g_a); out[a] receives the post-collision value in
// the same convention.
//   BGK (eq. eqLBEMCa): g* = g - (g - g_eq)/tau + (1 - 1/(2 tau)) F_a.
//   MRT: g* = g + F_a - M^-1 S M v with v = g - g_eq + F_a/2.  With an
//   orthogonal moment basis M^-1 S M = s_g I + sum_k (s_k - s_g) P_k over the
//   momentum, traceless-stress and energy groups (P_k the orthogonal projector
//   of group k); the conserved density row contributes nothing because
//   sum_a v_a = 0.
//   STD: the standard equilibrium w_a rho (1 + B_a) (every direction carries
//   w_a rho instead of the rest one carrying rho); the caller passes G = 0 so
//   the forcing is Guo's term without the grad rho part.
template <typename L, typename T, bool MRT, bool REST_OFFSET, bool STD = false>
__device__ __forceinline__ void collide(const KParams& kp, const CompState<T>& c, const T (&gv)[L::Q],
                                        T moving_sum, T (&out)[L::Q]) {
    constexpr int Q = L::Q;
    const T uu = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
    const T uF = c.ux * c.Fx + c.uy * c.Fy + c.uz * c.Fz;
    const T uG = c.ux * c.Gx + c.uy * c.Gy + c.uz * c.Gz;
    T neq[Q];  // g - g_eq
    T Fa[Q];
    Unroll<0, Q>::run([&](auto ai) {
        constexpr int a = decltype(ai)::value;
        const T sh = geq_shape<L, T, a>(c, uu);
        if constexpr (STD) {
            static_assert(!REST_OFFSET, "standard form: FP64 populations only");
            neq[a] = gv[a] - (T(L::w[a]) * c.rho + sh);
        } else if constexpr (a == 0) {
            if constexpr (REST_OFFSET)
                neq[0] = -moving_sum - sh;      // g_0 - rho - w_0 rho B_0
            else
                neq[0] = gv[0] - (c.rho + sh);
        } else {
            neq[a] = gv[a] - sh;
        }
        Fa[a] = forcing<L, T, a>(c, uF, uG);
    });
    if constexpr (!MRT) {
        const T om = T(kp.omega), cf = T(kp.cF);
#pragma unroll
        for (int a = 0; a < Q; ++a) out[a] = gv[a] - om * neq[a] + cf * Fa[a];
    } else {
        const T sg = T(kp.s_g);
        T v[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) v[a] = neq[a] + T(0.5) * Fa[a];
        // group moments of v
        T jx = 0, jy = 0, jz = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0, me = 0;
        Unroll<0, Q>::run([&](auto ai) {
            constexpr int a = decltype(ai)::value;
            constexpr T ex = L::ex[a], ey = L::ey[a], ez = L::ez[a];
            constexpr T e2 = ex * ex + ey * ey + ez * ez;
            jx += ex * v[a];
            jy += ey * v[a];
            jz += ez * v[a];
            if constexpr (L::D == 2) {
                m1 += (ex * ex - ey * ey) * v[a];
                m2 += (ex * ey) * v[a];
                me += (T(-4) + T(3) * e2) * v[a];
            } else {
                m1 += (T(3) * ex * ex - e2) * v[a];
                m2 += (ey * ey - ez * ez) * v[a];
                m3 += (ex * ey) * v[a];
                m4 += (ey * ez) * v[a];
                m5 += (ex * ez) * v[a];
                me += (T(19) * e2 - T(30)) * v[a];
            }
        });
        // scale by (s_k - s_g) / |row|^2 (per-launch constants)
        if constexpr (L::D == 2) {
            jx *= T(kp.mrt_f[0]); jy *= T(kp.mrt_f[1]);
            m1 *= T(kp.mrt_f[2]); m2 *= T(kp.mrt_f[3]);
            me *= T(kp.mrt_f[4]);
        } else {
            jx *= T(kp.mrt_f[0]); jy *= T(kp.mrt_f[1]); jz *= T(kp.mrt_f[2]);
            m1 *= T(kp.mrt_f[3]); m2 *= T(kp.mrt_f[4]); m3 *= T(kp.mrt_f[5]); m4 *= T(kp.mrt_f[6]);
            m5 *= T(kp.mrt_f[7]);
            me *= T(kp.mrt_f[8]);
        }
        Unroll<0, Q>::run([&](auto ai) {
            constexpr int a = decltype(ai)::value;
            constexpr T ex = L::ex[a], ey = L::ey[a], ez = L::ez[a];
            constexpr T e2 = ex * ex + ey * ey + ez * ez;
            T corr = ex * jx + ey * jy + ez * jz;
            if constexpr (L::D == 2) {
                corr += (ex * ex - ey * ey) * m1 + (ex * ey) * m2 + (T(-4) + T(3) * e2) * me;
            } else {
                corr += (T(3) * ex * ex - e2) * m1 + (ey * ey - ez * ez) * m2 + (ex * ey) * m3 +
                        (ey * ez) * m4 + (ex * ez) * m5 + (T(19) * e2 - T(30)) * me;
            }
            out[a] = gv[a] + Fa[a] - sg * v[a] - corr;
        });
    }
}

// The same collision over opposite pairs (a, a + 1), e_{a+1} = -e_a (how the
// lattices store their directions): over a pair the equilibrium shape and the
// forcing split into a part even in e (the same for both) and an odd one
// (opposite signs),
//   shape   w rho (9/2 (e.u)^2 - 3/2 u.u)  +-  3 w rho (e.u),
//   forcing w ((e.u)(9 e.F + 3 e.G) - 3 u.F + h u.G)  +-  3 w (e.F),
// h = -1 + (3 e^2 - D)/2, and the MRT group moments take the odd ones (the
// momentum) from v_a - v_{a+1} and the even ones (stress, energy) from
// v_a + v_{a+1}; the correction of direction a + 1 is the even part minus the
// odd one.  Algebraically the same, about a third fewer operations; other
// rounding.
template <typename L, typename T, int A>
struct PairDir {
    static constexpr T ex = L::ex[A], ey = L::ey[A], ez = L::ez[A];
    static constexpr T e2 = ex * ex + ey * ey + ez * ez;
    static_assert(L::ex[A + 1] == -L::ex[A] && L::ey[A + 1] == -L::ey[A] && L::ez[A + 1] == -L::ez[A],
                  "directions stored in opposite pairs");
};

template <typename L, typename T, bool MRT, bool REST_OFFSET, bool STD = false>
__device__ __forceinline__ void collide_pairs(const KParams& kp, const CompState<T>& c, const T (&gv)[L::Q],
                                              T moving_sum, T (&out)[L::Q]) {
    constexpr int NP = (L::Q - 1) / 2;
    const T uu = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
    const T uF = c.ux * c.Fx + c.uy * c.Fy + c.uz * c.Fz;
    const T uG = c.ux * c.Gx + c.uy * c.Gy + c.uz * c.Gz;
    const T su = T(-1.5) * uu;
    // rest direction: e = 0
    constexpr T h0 = T(-1) + T(0.5) * (T(0) - T(L::D));
    const T sh0 = T(L::w[0]) * c.rho * su;
    const T F0 = T(L::w[0]) * (T(-3) * uF + h0 * uG);
    T neq0;
    if constexpr (STD) {
        static_assert(!REST_OFFSET, "standard form: FP64 populations only");
        neq0 = gv[0] - (T(L::w[0]) * c.rho + sh0);
    } else if constexpr (REST_OFFSET) {
        neq0 = -moving_sum - sh0;      // g_0 - rho - w_0 rho B_0
    } else {
        neq0 = gv[0] - (c.rho + sh0);
    }
    // pairs: g - g_eq of both directions, even and odd parts of the forcing
    T na[NP], nb[NP], fE[NP], fO[NP];
    Unroll<0, NP>::run([&](auto pi) {
        constexpr int p = decltype(pi)::value;
        constexpr int a = 1 + 2 * p;
        using E = PairDir<L, T, a>;
        constexpr T h = T(-1) + T(0.5) * (T(3) * E::e2 - T(L::D));
        const T wr = T(L::w[a]) * c.rho;
        const T eu = E::ex * c.ux + E::ey * c.uy + E::ez * c.uz;
        const T eF = E::ex * c.Fx + E::ey * c.Fy + E::ez * c.Fz;
        const T eG = E::ex * c.Gx + E::ey * c.Gy + E::ez * c.Gz;
        T shE = wr * (T(4.5) * eu * eu + su);
        if constexpr (STD) shE += wr;
        const T shO = T(3) * wr * eu;
        fE[p] = T(L::w[a]) * (eu * (T(9) * eF + T(3) * eG) + (T(-3) * uF + h * uG));
        fO[p] = T(3) * T(L::w[a]) * eF;
        na[p] = gv[a] - (shE + shO);
        nb[p] = gv[a + 1] - (shE - shO);
    });
    if constexpr (!MRT) {
        const T om = T(kp.omega), cf = T(kp.cF);
        out[0] = gv[0] - om * neq0 + cf * F0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int a = 1 + 2 * p;
            out[a] = gv[a] - om * na[p] + cf * (fE[p] + fO[p]);
            out[a + 1] = gv[a + 1] - om * nb[p] + cf * (fE[p] - fO[p]);
        }
    } else {
        const T sg = T(kp.s_g);
        const T v0 = neq0 + T(0.5) * F0;
        T va[NP], vb[NP];
        T jx = 0, jy = 0, jz = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0, me = 0;
        Unroll<0, NP>::run([&](auto pi) {
            constexpr int p = decltype(pi)::value;
            using E = PairDir<L, T, 1 + 2 * p>;
            va[p] = na[p] + T(0.5) * (fE[p] + fO[p]);
            vb[p] = nb[p] + T(0.5) * (fE[p] - fO[p]);
            const T ve = va[p] + vb[p], vo = va[p] - vb[p];   // even and odd parts
            if constexpr (E::ex != 0) jx += E::ex * vo;
            if constexpr (E::ey != 0) jy += E::ey * vo;
            if constexpr (E::ez != 0) jz += E::ez * vo;
            if constexpr (L::D == 2) {
                if constexpr (E::ex * E::ex - E::ey * E::ey != 0) m1 += (E::ex * E::ex - E::ey * E::ey) * ve;
                if constexpr (E::ex * E::ey != 0) m2 += (E::ex * E::ey) * ve;
                me += (T(-4) + T(3) * E::e2) * ve;
            } else {
                if constexpr (T(3) * E::ex * E::ex - E::e2 != 0) m1 += (T(3) * E::ex * E::ex - E::e2) * ve;
                if constexpr (E::ey * E::ey - E::ez * E::ez != 0) m2 += (E::ey * E::ey - E::ez * E::ez) * ve;
                if constexpr (E::ex * E::ey != 0) m3 += (E::ex * E::ey) * ve;
                if constexpr (E::ey * E::ez != 0) m4 += (E::ey * E::ez) * ve;
                if constexpr (E::ex * E::ez != 0) m5 += (E::ex * E::ez) * ve;
                me += (T(19) * E::e2 - T(30)) * ve;
            }
        });
        constexpr T erest = L::D == 2 ? T(-4) : T(-30);   // energy row of the rest direction
        me += erest * v0;
        if constexpr (L::D == 2) {
            jx *= T(kp.mrt_f[0]); jy *= T(kp.mrt_f[1]);
            m1 *= T(kp.mrt_f[2]); m2 *= T(kp.mrt_f[3]);
            me *= T(kp.mrt_f[4]);
        } else {
            jx *= T(kp.mrt_f[0]); jy *= T(kp.mrt_f[1]); jz *= T(kp.mrt_f[2]);
            m1 *= T(kp.mrt_f[3]); m2 *= T(kp.mrt_f[4]); m3 *= T(kp.mrt_f[5]); m4 *= T(kp.mrt_f[6]);
            m5 *= T(kp.mrt_f[7]);
            me *= T(kp.mrt_f[8]);
        }
        out[0] = gv[0] + F0 - sg * v0 - erest * me;
        Unroll<0, NP>::run([&](auto pi) {
            constexpr int p = decltype(pi)::value;
            constexpr int a = 1 + 2 * p;
            using E = PairDir<L, T, a>;
            T co = 0, ce = 0;
            if constexpr (E::ex != 0) co += E::ex * jx;
            if constexpr (E::ey != 0) co += E::ey * jy;
            if constexpr (E::ez != 0) co += E::ez * jz;
            if constexpr (L::D == 2) {
                if constexpr (E::ex * E::ex - E::ey * E::ey != 0) ce += (E::ex * E::ex - E::ey * E::ey) * m1;
                if constexpr (E::ex * E::ey != 0) ce += (E::ex * E::ey) * m2;
                ce += (T(-4) + T(3) * E::e2) * me;
            } else {
                if constexpr (T(3) * E::ex * E::ex - E::e2 != 0) ce += (T(3) * E::ex * E::ex - E::e2) * m1;
                if constexpr (E::ey * E::ey - E::ez * E::ez != 0) ce += (E::ey * E::ey - E::ez * E::ez) * m2;
                if constexpr (E::ex * E::ey != 0) ce += (E::ex * E::ey) * m3;
                if constexpr (E::ey * E::ez != 0) ce += (E::ey * E::ez) * m4;
                if constexpr (E::ex * E::ez != 0) ce += (E::ex * E::ez) * m5;
                ce += (T(19) * E::e2 - T(30)) * me;
            }
            out[a] = gv[a] + (fE[p] + fO[p]) - sg * va[p] - (ce + co);
            out[a + 1] = gv[a + 1] + (fE[p] - fO[p]) - sg * vb[p] - (ce - co);
        });
    }
}

}  // namespace fl
