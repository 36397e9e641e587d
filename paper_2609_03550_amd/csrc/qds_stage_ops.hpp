// Field accessors of the staged step (boundary rules of the staggered grid)
// and the per-mode factors of the axion current; shared by the staged
// kernels and their adjoints.
#pragma once
#include "qds_kernels.hpp"

namespace qds {

// ---------------------------------------------------------------------------
// accessors with the x boundary rule: value at integer column c, zero beyond
// the ends unless x is periodic
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cx<T> ldx(const cx<T>* p, const Geo& g, int m, int row, int c) {
    if (c < 0 || c >= g.nx) {
        if (!g.per) return zero<T>();
        c = (c + g.nx) % g.nx;
    }
    return ld(p + g.at(m, row, c));
}

// B_theta at (x_c, r_{k+1/2}) from T_r, with row nr the stored exterior ghost
template <typename T>
__device__ __forceinline__ cx<T> bth(const SetPtr<T>& s, const Geo& g, int m, int k, int c) {
    if (k == g.nr) return ldx(s.trp, g, m, k, c);
    return T(0.5) * (ldx(s.trp, g, m, k, c) - ldx(s.trm, g, m, k, c));
}
template <typename T>
__device__ __forceinline__ cx<T> er(const SetPtr<T>& s, const Geo& g, int m, int k, int c) {
    return T(0.5) * (ldx(s.trp, g, m, k, c) + ldx(s.trm, g, m, k, c));
}
template <typename T>
__device__ __forceinline__ cx<T> eth(const SetPtr<T>& s, const Geo& g, int m, int j, int c) {
    return T(0.5) * (ldx(s.ttp, g, m, j, c) + ldx(s.ttm, g, m, j, c));
}
template <typename T>
__device__ __forceinline__ cx<T> brr(const SetPtr<T>& s, const Geo& g, int m, int j, int c) {
    return T(0.5) * (ldx(s.ttp, g, m, j, c) - ldx(s.ttm, g, m, j, c));
}

template <typename T>
struct BgView {
    // background fields around one point, built from A (time n) and B (n+1)
    const AxionArgs<T>* a;
    __device__ cx<T> Er0(int m, int k, int c) const { return er(a->A0, a->g, m, k, c); }
    __device__ cx<T> Bt0(int m, int k, int c) const { return bth(a->A0, a->g, m, k, c); }
    __device__ cx<T> Et0(int m, int j, int c) const { return eth(a->A0, a->g, m, j, c); }
    __device__ cx<T> Br0(int m, int j, int c) const { return brr(a->A0, a->g, m, j, c); }
    __device__ cx<T> Er1(int m, int k, int c) const { return er(a->B0, a->g, m, k, c); }
    __device__ cx<T> Bt1(int m, int k, int c) const {
        return T(0.5) * (ldx(a->B0.trp, a->g, m, k, c) - ldx(a->B0.trm, a->g, m, k, c));
    }
    __device__ cx<T> Et1(int m, int j, int c) const { return eth(a->B0, a->g, m, j, c); }
    __device__ cx<T> Br1(int m, int j, int c) const { return brr(a->B0, a->g, m, j, c); }
    // d_t phi and d_x phi from T_a at t^{n-1/2} (old) and t^{n+1/2} (new)
    __device__ cx<T> dto(int m, int k, int c) const {
        return T(0.5) * (ldx(a->tapA, a->g, m, k, c) + ldx(a->tamA, a->g, m, k, c));
    }
    __device__ cx<T> dth(int m, int k, int c) const {
        return T(0.5) * (ldx(a->tapB, a->g, m, k, c) + ldx(a->tamB, a->g, m, k, c));
    }
    __device__ cx<T> dxh(int m, int k, int c) const {
        return T(0.5) * (ldx(a->tamB, a->g, m, k, c) - ldx(a->tapB, a->g, m, k, c));
    }
};

// The 18 per-mode factors of the axion current at H cell i, row j < nr (each
// component is sum over three C_m{A, B} with signs +, -, +):
//   f[0..5]   j_a,x     at (x_{i+1/2}, r_j,       t^n):       B_x, d_t phi | E_r, (d_theta phi)/r | E_theta, d_r phi
//   f[6..11]  j_a,theta at (x_{i+1/2}, r_j,       t^{n+1/2}): B_theta, d_t phi | E_x, d_r phi | E_r, d_x phi
//   f[12..17] j_a,r     at (x_{i+1/2}, r_{j+1/2}, t^{n+1/2}): B_r, d_t phi | E_theta, d_x phi | E_x, (d_theta phi)/r
// Off-grid values are centred means of the nearest samples, with the axis
// reflections (parity (-1)^m for B_x, phi, T_a; (-1)^(m-1) for E_r and
// B_theta, whose mode 1 takes the axis relation); the uniform external field is
// added to the B factors.
//
// With TFORM the theta and r pairs are formed from the transport variables
// instead (same value in exact arithmetic, by bilinearity and symmetry of C_m):
//   C{B_th, d_t phi} + C{E_r, d_x phi} = 1/2 C{T_r^+, T_a^-} - 1/2 C{T_r^-, T_a^+}
//   C{B_r, d_t phi} - C{E_th, d_x phi} = 1/2 C{T_th^+, T_a^+} - 1/2 C{T_th^-, T_a^-}
// (T_a^+- = d_t phi -+ d_x phi; the external field enters as T_r^+- +- b_th,
// T_th^+- +- b_r).  For co-propagating waves each product then pairs a large
// factor with a small one, where the E/B form subtracts two large products;
// the single-precision forward uses it for that reason.
// PART selects one component's six factors (0: j_a,x into f[0..5],
// 1: j_a,theta into f[6..11], 2: j_a,r into f[12..17]); -1 forms all 18.
template <typename T, bool TFORM = false, int PART = -1>
__device__ void ja_factors(const AxionArgs<T>& a, int m, int i, int j, cx<T>* f) {
    const Geo& g = a.g;
    BgView<T> v{&a};
    const T dr = T(g.dr);
    const int i1 = i + 1;
    const bool ax = (j == 0);
    const T rj = T(j) * dr;
    const T rk = (T(j) + T(0.5)) * dr;
    const T r_half = T(0.5) * dr;
    const T par = parity<T>(m);
    const T tg = tghost<T>(m);
    // ---------------- j_a,x
    if constexpr (PART < 0 || PART == 0) {
        cx<T> bhi = T(0.5) * (ld(a.A0.bx + g.at(m, j, i)) + ld(a.B0.bx + g.at(m, j, i)));
        cx<T> blo = ax ? par * bhi : T(0.5) * (ld(a.A0.bx + g.at(m, j - 1, i)) + ld(a.B0.bx + g.at(m, j - 1, i)));
        f[0] = T(0.5) * (blo + bhi);
        if (m == 0) f[0] = f[0] + a.bx0;
        cx<T> d0 = T(0.5) * (v.dto(m, j, i) + v.dth(m, j, i));
        cx<T> d1 = T(0.5) * (v.dto(m, j, i1) + v.dth(m, j, i1));
        cx<T> l0 = ax ? par * d0 : T(0.5) * (v.dto(m, j - 1, i) + v.dth(m, j - 1, i));
        cx<T> l1 = ax ? par * d1 : T(0.5) * (v.dto(m, j - 1, i1) + v.dth(m, j - 1, i1));
        f[1] = T(0.5) * (T(0.5) * (l0 + d0) + T(0.5) * (l1 + d1));
        cx<T> e0 = v.Er0(m, j, i), e1 = v.Er0(m, j, i1);
        cx<T> g0, g1;
        if (ax) {
            if (m == 1) {
                g0 = imul(T(2), v.Et0(1, 0, i)) - e0;
                g1 = imul(T(2), v.Et0(1, 0, i1)) - e1;
            } else {
                g0 = tg * e0;
                g1 = tg * e1;
            }
        } else {
            g0 = v.Er0(m, j - 1, i);
            g1 = v.Er0(m, j - 1, i1);
        }
        f[2] = T(0.5) * (T(0.5) * (g0 + e0) + T(0.5) * (g1 + e1));
        cx<T> phi_hi = ld(a.phiA + g.at(m, j, i));
        cx<T> phi_lo = ax ? par * phi_hi : ld(a.phiA + g.at(m, j - 1, i));
        if (ax) f[3] = (m == 1) ? imul(-T(1) / r_half, phi_hi) : zero<T>();
        else f[3] = imul(-T(m) / rj, T(0.5) * (phi_lo + phi_hi));
        f[4] = T(0.5) * (v.Et0(m, j, i) + v.Et0(m, j, i1));
        f[5] = (T(1) / dr) * (phi_hi - phi_lo);
    }
    // ---------------- j_a,theta
    if constexpr (PART >= 0 && PART != 1) {
    } else if constexpr (TFORM) {
        // T_r^+- averaged over t^n, t^{n+1} at (i or i1, j+1/2)
        auto tr = [&](const cx<T>* p0, const cx<T>* p1, int k, int c) {
            return T(0.5) * (ldx(p0, g, m, k, c) + ldx(p1, g, m, k, c));
        };
        cx<T> P0 = tr(a.A0.trp, a.B0.trp, j, i), P1 = tr(a.A0.trp, a.B0.trp, j, i1);
        cx<T> N0 = tr(a.A0.trm, a.B0.trm, j, i), N1 = tr(a.A0.trm, a.B0.trm, j, i1);
        cx<T> gP0, gP1, gN0, gN1;
        if (ax) {
            if (m == 1) {
                // E_r, B_theta ghosts of the m = 1 axis relation, combined:
                // T_r^+ ghost = 2i T_th^-(0) - T_r^+(1/2), T_r^- ghost = 2i T_th^+(0) - T_r^-(1/2)
                auto tt = [&](const cx<T>* p0, const cx<T>* p1, int c) {
                    return T(0.5) * (ldx(p0, g, 1, 0, c) + ldx(p1, g, 1, 0, c));
                };
                gP0 = imul(T(2), tt(a.A0.ttm, a.B0.ttm, i)) - P0;
                gP1 = imul(T(2), tt(a.A0.ttm, a.B0.ttm, i1)) - P1;
                gN0 = imul(T(2), tt(a.A0.ttp, a.B0.ttp, i)) - N0;
                gN1 = imul(T(2), tt(a.A0.ttp, a.B0.ttp, i1)) - N1;
            } else {
                gP0 = tg * P0; gP1 = tg * P1; gN0 = tg * N0; gN1 = tg * N1;
            }
        } else {
            gP0 = tr(a.A0.trp, a.B0.trp, j - 1, i);
            gP1 = tr(a.A0.trp, a.B0.trp, j - 1, i1);
            gN0 = tr(a.A0.trm, a.B0.trm, j - 1, i);
            gN1 = tr(a.A0.trm, a.B0.trm, j - 1, i1);
        }
        cx<T> fP = T(0.5) * (T(0.5) * (gP0 + P0) + T(0.5) * (gP1 + P1));
        cx<T> fN = T(0.5) * (T(0.5) * (gN0 + N0) + T(0.5) * (gN1 + N1));
        if (m == 1) { fP = fP + a.bt1; fN = fN - a.bt1; }
        const cx<T>* tpB = a.tapB;
        const cx<T>* tmB = a.tamB;
        cx<T> u0 = ldx(tpB, g, m, j, i), u1 = ldx(tpB, g, m, j, i1);
        cx<T> w0 = ldx(tmB, g, m, j, i), w1 = ldx(tmB, g, m, j, i1);
        cx<T> ul0 = ax ? par * u0 : ldx(tpB, g, m, j - 1, i), ul1 = ax ? par * u1 : ldx(tpB, g, m, j - 1, i1);
        cx<T> wl0 = ax ? par * w0 : ldx(tmB, g, m, j - 1, i), wl1 = ax ? par * w1 : ldx(tmB, g, m, j - 1, i1);
        f[6] = T(0.5) * fP;
        f[7] = T(0.5) * (T(0.5) * (wl0 + w0) + T(0.5) * (wl1 + w1));      // T_a^-
        f[10] = T(-0.5) * fN;
        f[11] = T(0.5) * (T(0.5) * (ul0 + u0) + T(0.5) * (ul1 + u1));     // T_a^+
        f[8] = ld(a.B0.ex + g.at(m, j, i));
        cx<T> ph = T(0.5) * (ld(a.phiA + g.at(m, j, i)) + ld(a.phiB + g.at(m, j, i)));
        cx<T> pl = ax ? par * ph : T(0.5) * (ld(a.phiA + g.at(m, j - 1, i)) + ld(a.phiB + g.at(m, j - 1, i)));
        f[9] = (T(1) / dr) * (ph - pl);
    } else {
        cx<T> b0 = T(0.5) * (v.Bt0(m, j, i) + v.Bt1(m, j, i));
        cx<T> b1 = T(0.5) * (v.Bt0(m, j, i1) + v.Bt1(m, j, i1));
        cx<T> e0 = T(0.5) * (v.Er0(m, j, i) + v.Er1(m, j, i));
        cx<T> e1 = T(0.5) * (v.Er0(m, j, i1) + v.Er1(m, j, i1));
        cx<T> gb0, gb1, ge0, ge1;
        if (ax) {
            if (m == 1) {
                cx<T> br0 = T(0.5) * (v.Br0(1, 0, i) + v.Br1(1, 0, i));
                cx<T> br1 = T(0.5) * (v.Br0(1, 0, i1) + v.Br1(1, 0, i1));
                cx<T> et0 = T(0.5) * (v.Et0(1, 0, i) + v.Et1(1, 0, i));
                cx<T> et1 = T(0.5) * (v.Et0(1, 0, i1) + v.Et1(1, 0, i1));
                gb0 = imul(-T(2), br0) - b0;
                gb1 = imul(-T(2), br1) - b1;
                ge0 = imul(T(2), et0) - e0;
                ge1 = imul(T(2), et1) - e1;
            } else {
                gb0 = tg * b0; gb1 = tg * b1; ge0 = tg * e0; ge1 = tg * e1;
            }
        } else {
            gb0 = T(0.5) * (v.Bt0(m, j - 1, i) + v.Bt1(m, j - 1, i));
            gb1 = T(0.5) * (v.Bt0(m, j - 1, i1) + v.Bt1(m, j - 1, i1));
            ge0 = T(0.5) * (v.Er0(m, j - 1, i) + v.Er1(m, j - 1, i));
            ge1 = T(0.5) * (v.Er0(m, j - 1, i1) + v.Er1(m, j - 1, i1));
        }
        f[6] = T(0.5) * (T(0.5) * (gb0 + b0) + T(0.5) * (gb1 + b1));
        if (m == 1) f[6] = f[6] + a.bt1;
        f[10] = T(0.5) * (T(0.5) * (ge0 + e0) + T(0.5) * (ge1 + e1));
        cx<T> t0 = v.dth(m, j, i), t1 = v.dth(m, j, i1);
        cx<T> x0 = v.dxh(m, j, i), x1 = v.dxh(m, j, i1);
        cx<T> tl0 = ax ? par * t0 : v.dth(m, j - 1, i), tl1 = ax ? par * t1 : v.dth(m, j - 1, i1);
        cx<T> xl0 = ax ? par * x0 : v.dxh(m, j - 1, i), xl1 = ax ? par * x1 : v.dxh(m, j - 1, i1);
        f[7] = T(0.5) * (T(0.5) * (tl0 + t0) + T(0.5) * (tl1 + t1));
        f[11] = T(0.5) * (T(0.5) * (xl0 + x0) + T(0.5) * (xl1 + x1));
        f[8] = ld(a.B0.ex + g.at(m, j, i));
        cx<T> ph = T(0.5) * (ld(a.phiA + g.at(m, j, i)) + ld(a.phiB + g.at(m, j, i)));
        cx<T> pl = ax ? par * ph : T(0.5) * (ld(a.phiA + g.at(m, j - 1, i)) + ld(a.phiB + g.at(m, j - 1, i)));
        f[9] = (T(1) / dr) * (ph - pl);
    }
    // ---------------- j_a,r
    if constexpr (PART >= 0 && PART != 2) {
    } else if constexpr (TFORM) {
        cx<T> sp = zero<T>(), sm = zero<T>();
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                sp = sp + T(0.5) * (ldx(a.A0.ttp, g, m, j + dj, i + di) + ldx(a.B0.ttp, g, m, j + dj, i + di));
                sm = sm + T(0.5) * (ldx(a.A0.ttm, g, m, j + dj, i + di) + ldx(a.B0.ttm, g, m, j + dj, i + di));
            }
        cx<T> qp = T(0.25) * sp, qm = T(0.25) * sm;
        if (m == 1) { qp = qp + a.br1; qm = qm - a.br1; }
        f[12] = T(0.5) * qp;
        f[13] = T(0.5) * (ldx(a.tapB, g, m, j, i) + ldx(a.tapB, g, m, j, i1));   // T_a^+
        f[14] = T(0.5) * qm;
        f[15] = T(0.5) * (ldx(a.tamB, g, m, j, i) + ldx(a.tamB, g, m, j, i1));   // T_a^-
        f[16] = T(0.5) * (ld(a.B0.ex + g.at(m, j, i)) + ld(a.B0.ex + g.at(m, j + 1, i)));
        cx<T> ph = T(0.5) * (ld(a.phiA + g.at(m, j, i)) + ld(a.phiB + g.at(m, j, i)));
        f[17] = imul(-T(m) / rk, ph);
    } else {
        cx<T> sb = zero<T>(), se = zero<T>();
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                sb = sb + T(0.5) * (v.Br0(m, j + dj, i + di) + v.Br1(m, j + dj, i + di));
                se = se + T(0.5) * (v.Et0(m, j + dj, i + di) + v.Et1(m, j + dj, i + di));
            }
        f[12] = T(0.25) * sb;
        if (m == 1) f[12] = f[12] + a.br1;
        f[13] = T(0.5) * (v.dth(m, j, i) + v.dth(m, j, i1));
        f[14] = T(0.25) * se;
        f[15] = T(0.5) * (v.dxh(m, j, i) + v.dxh(m, j, i1));
        f[16] = T(0.5) * (ld(a.B0.ex + g.at(m, j, i)) + ld(a.B0.ex + g.at(m, j + 1, i)));
        cx<T> ph = T(0.5) * (ld(a.phiA + g.at(m, j, i)) + ld(a.phiB + g.at(m, j, i)));
        f[17] = imul(-T(m) / rk, ph);
    }
}

}  // namespace qds
