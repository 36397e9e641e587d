// Row windows and per-mode factors of the marched axion current (Eqs.
// jax_mode, jar_mode, jat_mode in the transport-variable form), shared by the
// forward march and its adjoint so that both evaluate the same expressions.
//
// A lane holds column i of one mode; a half row K = j carries the per-point
// combinations of the old (A) and new (B) background set, axion and T_a that
// the factors read, an integer row J = j those of T_theta and E_x.  Values of
// column i+1 come from the next lane.  The adjoint loads a K row with load_k
// (the new axion values from the recomputed state); the forward march forms
// the new T_a and phi of the row itself.
#pragma once
#include "qds_kernels.hpp"

namespace qds {
namespace cur {

constexpr int WAVE = 64;

template <typename T>
__device__ __forceinline__ uint32_t eoff(const Geo& g, int m, int row, int c) {
    return (uint32_t(m * (g.nr + 1) + row) * uint32_t(g.ld) + uint32_t(c)) * uint32_t(sizeof(cx<T>));
}
typedef __attribute__((address_space(1))) const char g_cchar;
typedef __attribute__((address_space(1))) char g_char;
template <typename T>
__device__ __forceinline__ cx<T> ldo(const cx<T>* p, uint32_t o) {
    return ld((const cx<T>*)((g_cchar*)(p) + o));
}
template <typename T>
__device__ __forceinline__ void sto(cx<T>* p, uint32_t o, cx<T> v) {
    st((cx<T>*)((g_char*)(p) + o), v);
}

// per-point quantities on a half row K (at column i of the lane)
template <typename T>
struct KRow {
    cx<T> bxn;    // B_x at t^n (mean of t^{n-1/2}, t^{n+1/2})
    cx<T> dt0;    // d_t phi at t^n (mean of T_a-sums at t^{n-1/2}, t^{n+1/2})
    cx<T> er0;    // E_r at t^n
    cx<T> ph0;    // phi^n
    cx<T> P, N;   // T_r^+, T_r^- averaged over t^n, t^{n+1}
    cx<T> up, wm; // T_a^+, T_a^- at t^{n+1/2}
    cx<T> phm;    // phi averaged over t^n, t^{n+1}
};
// per-point quantities on an integer row J
template <typename T>
struct JRow {
    cx<T> et0;    // E_theta at t^n
    cx<T> ex;     // E_x at t^{n+1/2}
    cx<T> Qp, Qm; // T_theta^+, T_theta^- averaged over t^n, t^{n+1}
};

template <typename T>
__device__ __forceinline__ KRow<T> load_k(const AxionArgs<T>& a, uint32_t o) {
    KRow<T> r;
    const T q = T(0.5);
    r.bxn = q * (ldo(a.A0.bx, o) + ldo(a.B0.bx, o));
    const cx<T> tpA = ldo(a.tapA, o), tmA = ldo(a.tamA, o);
    r.up = ldo(a.tapB, o);
    r.wm = ldo(a.tamB, o);
    r.dt0 = q * (q * (tpA + tmA) + q * (r.up + r.wm));
    const cx<T> rpA = ldo(a.A0.trp, o), rmA = ldo(a.A0.trm, o);
    r.er0 = q * (rpA + rmA);
    r.P = q * (rpA + ldo(a.B0.trp, o));
    r.N = q * (rmA + ldo(a.B0.trm, o));
    r.ph0 = ldo(a.phiA, o);
    r.phm = q * (r.ph0 + ldo(a.phiB, o));
    return r;
}
template <typename T>
__device__ __forceinline__ JRow<T> load_j(const AxionArgs<T>& a, uint32_t o) {
    JRow<T> r;
    const T q = T(0.5);
    const cx<T> tpA = ldo(a.A0.ttp, o), tmA = ldo(a.A0.ttm, o);
    r.et0 = q * (tpA + tmA);
    r.Qp = q * (tpA + ldo(a.B0.ttp, o));
    r.Qm = q * (tmA + ldo(a.B0.ttm, o));
    r.ex = ldo(a.B0.ex, o);
    return r;
}
template <typename T>
__device__ __forceinline__ KRow<T> zero_k() {
    KRow<T> r;
    r.bxn = r.dt0 = r.er0 = r.ph0 = r.P = r.N = r.up = r.wm = r.phm = zero<T>();
    return r;
}
template <typename T>
__device__ __forceinline__ JRow<T> zero_j() {
    JRow<T> r;
    r.et0 = r.ex = r.Qp = r.Qm = zero<T>();
    return r;
}

// column i+1 of a value: the shift runs on every lane (a DPP read from a lane
// masked off by a branch would return zero); the missing column is zeroed
template <typename T>
__device__ __forceinline__ cx<T> nx1(cx<T> v, bool has1) {
    const cx<T> w = next_lane(v);
    return has1 ? w : zero<T>();
}

// the column-i+1 values each component reads (kp: K row j-1, kc: K row j,
// jc: J row j, jn: J row j+1)
template <typename T>
struct NbX {
    cx<T> dt1, er1, et1, dtl1, erl1;   // kc.dt0, kc.er0, jc.et0, kp.dt0, kp.er0
};
template <typename T>
struct NbR {
    cx<T> Qp1, Qm1, Qpn1, Qmn1, up1, wm1;   // jc.Qp, jc.Qm, jn.Qp, jn.Qm, kc.up, kc.wm
};
template <typename T>
struct NbT {
    cx<T> P1, N1, up1, wm1, Pl1, Nl1, upl1, wml1, Qp1, Qm1;   // kc.*, kp.*, jc.Qp, jc.Qm
};
template <typename T>
__device__ __forceinline__ NbX<T> nb_x(const KRow<T>& kp, const KRow<T>& kc, const JRow<T>& jc, bool has1) {
    return NbX<T>{nx1(kc.dt0, has1), nx1(kc.er0, has1), nx1(jc.et0, has1), nx1(kp.dt0, has1), nx1(kp.er0, has1)};
}
template <typename T>
__device__ __forceinline__ NbR<T> nb_r(const KRow<T>& kc, const JRow<T>& jc, const JRow<T>& jn, bool has1) {
    return NbR<T>{nx1(jc.Qp, has1), nx1(jc.Qm, has1), nx1(jn.Qp, has1),
                  nx1(jn.Qm, has1), nx1(kc.up, has1), nx1(kc.wm, has1)};
}
template <typename T>
__device__ __forceinline__ NbT<T> nb_t(const KRow<T>& kp, const KRow<T>& kc, const JRow<T>& jc, bool has1) {
    return NbT<T>{nx1(kc.P, has1),  nx1(kc.N, has1),  nx1(kc.up, has1), nx1(kc.wm, has1), nx1(kp.P, has1),
                  nx1(kp.N, has1),  nx1(kp.up, has1), nx1(kp.wm, has1), nx1(jc.Qp, has1), nx1(jc.Qm, has1)};
}

// constants of one wave's mode
template <typename T>
struct FacC {
    int m;
    T par;              // axis parity of B_x, phi, T_a: (-1)^m
    T tg;               // coefficient of T_r(1/2) in its axis ghost: (-1)^(m-1), -1 for m = 1
    T dr, inv_dr;
    cx<T> bx0, br1, bt1;   // uniform external field
};

// j_a,x at (x_{i+1/2}, r_j, t^n): factor pairs (B_x, d_t phi), (E_r, d_theta phi / r),
// (E_theta, d_r phi)
template <typename T>
__device__ __forceinline__ void fac_x(const FacC<T>& c, int j, const KRow<T>& kp, const KRow<T>& kc,
                                      const JRow<T>& jc, const NbX<T>& n, cx<T>* f) {
    const bool ax = j == 0;
    const int m = c.m;
    const T par = c.par;
    cx<T> blo = ax ? par * kc.bxn : kp.bxn;
    f[0] = T(0.5) * (blo + kc.bxn);
    if (m == 0) f[0] = f[0] + c.bx0;
    cx<T> l0 = ax ? par * kc.dt0 : kp.dt0, l1 = ax ? par * n.dt1 : n.dtl1;
    f[1] = T(0.5) * (T(0.5) * (l0 + kc.dt0) + T(0.5) * (l1 + n.dt1));
    cx<T> g0, g1;
    if (ax) {
        if (m == 1) {
            g0 = imul(T(2), jc.et0) - kc.er0;
            g1 = imul(T(2), n.et1) - n.er1;
        } else {
            g0 = c.tg * kc.er0;
            g1 = c.tg * n.er1;
        }
    } else {
        g0 = kp.er0;
        g1 = n.erl1;
    }
    f[2] = T(0.5) * (T(0.5) * (g0 + kc.er0) + T(0.5) * (g1 + n.er1));
    cx<T> plo = ax ? par * kc.ph0 : kp.ph0;
    f[3] = ax ? ((m == 1) ? imul(-T(2) * c.inv_dr, kc.ph0) : zero<T>())
              : imul(-T(m) * c.inv_dr / T(j), T(0.5) * (plo + kc.ph0));
    f[4] = T(0.5) * (jc.et0 + n.et1);
    f[5] = c.inv_dr * (kc.ph0 - plo);
}

// j_a,r at (x_{i+1/2}, r_{j+1/2}, t^{n+1/2}): pairs (B_r, d_t phi), (E_theta, d_x phi),
// (E_x, d_theta phi / r), with the transverse fields as T_theta averages
template <typename T>
__device__ __forceinline__ void fac_r(const FacC<T>& c, int j, const KRow<T>& kc, const JRow<T>& jc,
                                      const JRow<T>& jn, const NbR<T>& n, cx<T>* f) {
    const int m = c.m;
    cx<T> qp = T(0.25) * ((jc.Qp + n.Qp1) + (jn.Qp + n.Qpn1));
    cx<T> qm = T(0.25) * ((jc.Qm + n.Qm1) + (jn.Qm + n.Qmn1));
    if (m == 1) { qp = qp + c.br1; qm = qm - c.br1; }
    const T irk = T(1) / ((T(j) + T(0.5)) * c.dr);
    f[0] = T(0.5) * qp;
    f[1] = T(0.5) * (kc.up + n.up1);
    f[2] = T(0.5) * qm;
    f[3] = T(0.5) * (kc.wm + n.wm1);
    f[4] = T(0.5) * (jc.ex + jn.ex);
    f[5] = imul(-T(m) * irk, kc.phm);
}

// j_a,theta at (x_{i+1/2}, r_j, t^{n+1/2}): pairs (B_theta, d_t phi), (E_x, d_r phi),
// (E_r, d_x phi), with the transverse fields as T_r averages
template <typename T>
__device__ __forceinline__ void fac_t(const FacC<T>& c, int j, const KRow<T>& kp, const KRow<T>& kc,
                                      const JRow<T>& jc, const NbT<T>& n, cx<T>* f) {
    const bool ax = j == 0;
    const int m = c.m;
    const T par = c.par;
    cx<T> gP0, gP1, gN0, gN1;
    if (ax) {
        if (m == 1) {
            // axis relation of mode 1 (T_r^+ ghost 2i T_th^-(0) - T_r^+(1/2), T_r^- ghost 2i T_th^+(0) - T_r^-(1/2))
            gP0 = imul(T(2), jc.Qm) - kc.P;
            gP1 = imul(T(2), n.Qm1) - n.P1;
            gN0 = imul(T(2), jc.Qp) - kc.N;
            gN1 = imul(T(2), n.Qp1) - n.N1;
        } else {
            gP0 = c.tg * kc.P; gP1 = c.tg * n.P1; gN0 = c.tg * kc.N; gN1 = c.tg * n.N1;
        }
    } else {
        gP0 = kp.P; gP1 = n.Pl1; gN0 = kp.N; gN1 = n.Nl1;
    }
    cx<T> fP = T(0.5) * (T(0.5) * (gP0 + kc.P) + T(0.5) * (gP1 + n.P1));
    cx<T> fN = T(0.5) * (T(0.5) * (gN0 + kc.N) + T(0.5) * (gN1 + n.N1));
    if (m == 1) { fP = fP + c.bt1; fN = fN - c.bt1; }
    cx<T> ul0 = ax ? par * kc.up : kp.up, ul1 = ax ? par * n.up1 : n.upl1;
    cx<T> wl0 = ax ? par * kc.wm : kp.wm, wl1 = ax ? par * n.wm1 : n.wml1;
    cx<T> pl = ax ? par * kc.phm : kp.phm;
    f[0] = T(0.5) * fP;
    f[1] = T(0.5) * (T(0.5) * (wl0 + kc.wm) + T(0.5) * (wl1 + n.wm1));
    f[2] = jc.ex;
    f[3] = c.inv_dr * (kc.phm - pl);
    f[4] = T(-0.5) * fN;
    f[5] = T(0.5) * (T(0.5) * (ul0 + kc.up) + T(0.5) * (ul1 + n.up1));
}

}  // namespace cur
}  // namespace qds
