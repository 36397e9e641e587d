// Axion current j_a at the source points of the regenerated set (Eqs.
// jax_mode, jar_mode, jat_mode), marched in r.
//
// A workgroup is M wavefronts (one per mode) over one strip of 64 columns (63
// owned; lane 63 only lends its column to lane 62) and a chunk of radial
// rows.  Each lane walks its rows upward keeping, for the half row K = j-1 and
// the integer row J = j, the handful of per-point combinations the factors
// use (time averages of T^+-, E_r and E_theta at t^n, d_t phi at t^n, ...), so
// every input plane is read once per step; the values of column i+1 come from
// the next lane by a DPP shift.  The 18 per-mode factors are exchanged through
// LDS between the waves (two barriers per row), and each wave evaluates C_m
// for its own mode.  The factors are those of ja_factors with
// the transport-variable form of the theta and r components.
#include "qds_kernels.hpp"

namespace qds {
namespace cur {

constexpr int WAVE = 64;
constexpr int OWN = 63;

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

template <typename T, int M>
__device__ __forceinline__ void current_body(const AxionArgs<T>& a, int strip, int chunk, int rows) {
    const Geo& g = a.g;
    const int m = threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    const int raw = strip * OWN + lane;
    // halo lanes wrap with periodic x and are clamped otherwise
    const int i = g.per ? raw % g.nx : min(raw, g.nx - 1);
    const bool owner = lane < OWN && raw < g.nx;
    const bool has1 = g.per || i + 1 < g.nx;      // column i+1 exists
    const bool live = g.per || i < g.nx - 1;
    const int r0 = chunk * rows;
    const int r1 = min(g.nr + 1, r0 + rows);
    const T par = m == 0 ? T(1) : T(-1);
    const T dr = T(g.dr);
    const T inv_dr = T(1) / dr;
    const T sj = T(a.s_j);
    const cx<T> zc = zero<T>();

    // factor exchange in two phases: j_a,x and j_a,r (12 factors), then j_a,theta (6)
    __shared__ cx<T> sm[12][M][WAVE];
    auto put = [&](int f, cx<T> v) { sm[f][m][lane] = v; };
    // out += sum over the np factor pairs from pair c0 on of +-C_m (pair sgn_pair negated)
    auto convs = [&](int c0, int np, cx<T>& out, int sgn_pair) {
        cx<T> A[M], B[M];
#pragma unroll
        for (int c = 0; c < np; ++c) {
#pragma unroll
            for (int k = 0; k < M; ++k) { A[k] = sm[2 * (c0 + c)][k][lane]; B[k] = sm[2 * (c0 + c) + 1][k][lane]; }
            conv_one<T, M>(A, B, m, out, (c == sgn_pair) ? T(-1) : T(1));
        }
    };

    // window: K row j-1, J row j (and the m = 1 axis values of J row 0)
    KRow<T> kp = r0 >= 1 ? load_k(a, eoff<T>(g, m, r0 - 1, i)) : zero_k<T>();
    JRow<T> jc = load_j(a, eoff<T>(g, m, r0, i));
    // column i+1 of a value: the shift runs on every lane (a DPP read from a
    // lane masked off by a branch would return zero); the missing column is
    // zeroed after it
    auto nx1 = [&](cx<T> v) {
        const cx<T> w = next_lane(v);
        return has1 ? w : zc;
    };
    for (int j = r0; j < r1; ++j) {
        const bool calc = live && j < g.nr;
        KRow<T> kc = j < g.nr ? load_k(a, eoff<T>(g, m, j, i)) : zero_k<T>();
        JRow<T> jn = j + 1 <= g.nr ? load_j(a, eoff<T>(g, m, j + 1, i)) : zero_j<T>();
        const bool ax = j == 0;
        const uint32_t o = eoff<T>(g, m, j, i);
        {
            // ------------ j_a,x at (x_{i+1/2}, r_j, t^n): B_x, d_t phi | E_r, d_theta phi / r | E_theta, d_r phi
            const cx<T> dt1 = nx1(kc.dt0), er1 = nx1(kc.er0), et1 = nx1(jc.et0);
            const cx<T> dtl1 = nx1(kp.dt0), erl1 = nx1(kp.er0);
            if (calc) {
                cx<T> blo = ax ? par * kc.bxn : kp.bxn;
                cx<T> f0 = T(0.5) * (blo + kc.bxn);
                if (m == 0) f0 = f0 + a.bx0;
                cx<T> l0 = ax ? par * kc.dt0 : kp.dt0, l1 = ax ? par * dt1 : dtl1;
                cx<T> f1 = T(0.5) * (T(0.5) * (l0 + kc.dt0) + T(0.5) * (l1 + dt1));
                cx<T> g0, g1;
                if (ax) {
                    if (m == 1) {
                        g0 = imul(T(2), jc.et0) - kc.er0;
                        g1 = imul(T(2), et1) - er1;
                    } else {
                        g0 = -kc.er0;
                        g1 = -er1;
                    }
                } else {
                    g0 = kp.er0;
                    g1 = erl1;
                }
                cx<T> f2 = T(0.5) * (T(0.5) * (g0 + kc.er0) + T(0.5) * (g1 + er1));
                cx<T> plo = ax ? par * kc.ph0 : kp.ph0;
                cx<T> f3 = ax ? ((m == 1) ? imul(-T(2) * inv_dr, kc.ph0) : zc)
                              : imul(-T(m) * inv_dr / T(j), T(0.5) * (plo + kc.ph0));
                cx<T> f4 = T(0.5) * (jc.et0 + et1);
                cx<T> f5 = inv_dr * (kc.ph0 - plo);
                put(0, f0); put(1, f1); put(2, f2); put(3, f3); put(4, f4); put(5, f5);
            }
        }
        {
            // ------------ j_a,r at (x_{i+1/2}, r_{j+1/2}, t^{n+1/2}) in transport form
            const cx<T> Qp1 = nx1(jc.Qp), Qm1 = nx1(jc.Qm), Qpn1 = nx1(jn.Qp), Qmn1 = nx1(jn.Qm);
            const cx<T> up1 = nx1(kc.up), wm1 = nx1(kc.wm);
            if (calc) {
                cx<T> qp = T(0.25) * ((jc.Qp + Qp1) + (jn.Qp + Qpn1));
                cx<T> qm = T(0.25) * ((jc.Qm + Qm1) + (jn.Qm + Qmn1));
                if (m == 1) { qp = qp + a.br1; qm = qm - a.br1; }
                const T irk = T(1) / ((T(j) + T(0.5)) * dr);
                put(6, T(0.5) * qp);
                put(7, T(0.5) * (kc.up + up1));
                put(8, T(0.5) * qm);
                put(9, T(0.5) * (kc.wm + wm1));
                put(10, T(0.5) * (jc.ex + jn.ex));
                put(11, imul(-T(m) * irk, kc.phm));
            }
        }
        __syncthreads();
        {
            cx<T> ox = zc, orr = zc;
            if (calc) {
                convs(0, 3, ox, 1);
                convs(3, 3, orr, 1);
            }
            if (owner) {
                sto(a.jax, o, sj * ox);
                if (j < g.nr) sto(a.jar, o, sj * orr);
            }
        }
        __syncthreads();
        {
            // ------------ j_a,theta at (x_{i+1/2}, r_j, t^{n+1/2}) in transport form
            const cx<T> P1 = nx1(kc.P), N1 = nx1(kc.N), up1 = nx1(kc.up), wm1 = nx1(kc.wm);
            const cx<T> Pl1 = nx1(kp.P), Nl1 = nx1(kp.N), upl1 = nx1(kp.up), wml1 = nx1(kp.wm);
            const cx<T> Qp1 = nx1(jc.Qp), Qm1 = nx1(jc.Qm);
            if (calc) {
                cx<T> gP0, gP1, gN0, gN1;
                if (ax) {
                    if (m == 1) {
                        // axis relation of mode 1 (T_r^+ ghost 2i T_th^-(0) - T_r^+(1/2), T_r^- ghost 2i T_th^+(0) - T_r^-(1/2))
                        gP0 = imul(T(2), jc.Qm) - kc.P;
                        gP1 = imul(T(2), Qm1) - P1;
                        gN0 = imul(T(2), jc.Qp) - kc.N;
                        gN1 = imul(T(2), Qp1) - N1;
                    } else {
                        gP0 = -kc.P; gP1 = -P1; gN0 = -kc.N; gN1 = -N1;
                    }
                } else {
                    gP0 = kp.P; gP1 = Pl1; gN0 = kp.N; gN1 = Nl1;
                }
                cx<T> fP = T(0.5) * (T(0.5) * (gP0 + kc.P) + T(0.5) * (gP1 + P1));
                cx<T> fN = T(0.5) * (T(0.5) * (gN0 + kc.N) + T(0.5) * (gN1 + N1));
                if (m == 1) { fP = fP + a.bt1; fN = fN - a.bt1; }
                cx<T> ul0 = ax ? par * kc.up : kp.up, ul1 = ax ? par * up1 : upl1;
                cx<T> wl0 = ax ? par * kc.wm : kp.wm, wl1 = ax ? par * wm1 : wml1;
                cx<T> pl = ax ? par * kc.phm : kp.phm;
                put(0, T(0.5) * fP);
                put(1, T(0.5) * (T(0.5) * (wl0 + kc.wm) + T(0.5) * (wl1 + wm1)));
                put(2, jc.ex);
                put(3, inv_dr * (kc.phm - pl));
                put(4, T(-0.5) * fN);
                put(5, T(0.5) * (T(0.5) * (ul0 + kc.up) + T(0.5) * (ul1 + up1)));
            }
        }
        __syncthreads();
        {
            cx<T> ot = zc;
            if (calc) convs(0, 3, ot, 1);
            if (owner) sto(a.jat, o, sj * ot);
        }
        kp = kc;
        jc = jn;
        __syncthreads();
    }
}

template <typename T, int M>
__global__ void __launch_bounds__(WAVE * M) k_batch_current_march(const AxionArgs<T>* __restrict__ args, BatchList L) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int k = batch_find(L, b);
    const AxionArgs<T>& a = args[L.idx[k]];
    const int local = b - L.first[k];
    const int chunks = (a.g.nr + 1 + L.rows - 1) / L.rows;
    current_body<T, M>(a, local / chunks, local % chunks, L.rows);
}

}  // namespace cur

int current_strips(int nx) { return (nx + cur::OWN - 1) / cur::OWN; }

template <typename T>
hipError_t batch_current(const AxionArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    switch (M) {
#define QDS_BC(MM)                                                                                          \
    case MM:                                                                                                \
        hipLaunchKernelGGL((cur::k_batch_current_march<T, MM>), dim3(blocks), dim3(cur::WAVE * MM), 0, s, args, L); \
        break;
        QDS_BC(1) QDS_BC(2) QDS_BC(3) QDS_BC(4)
#undef QDS_BC
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t batch_current<double>(const AxionArgs<double>*, const BatchList&, int, int, hipStream_t);
template hipError_t batch_current<float>(const AxionArgs<float>*, const BatchList&, int, int, hipStream_t);

}  // namespace qds
