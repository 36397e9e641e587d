// Axion advance (Eqs. Ta_plus/minus_update, phi_update) and the axion current
// j_a at the source points of the regenerated set (Eqs. jax_mode, jar_mode,
// jat_mode), marched in r.
//
// A workgroup is M wavefronts (one per mode) over one strip of 64 columns (61
// owned; lane 0 a left halo, lanes 62-63 a right halo, as kernel A) and a
// chunk of radial rows.  Each lane walks its rows upward keeping, for the half
// row K = j-1 and the integer row J = j, the handful of per-point combinations
// the factors use (time averages of T^+-, E_r and E_theta at t^n, d_t phi at
// t^n, ...), so every input plane is read once per step; the values of column
// i+1 come from the next lane by a DPP shift.  On each half row the lane first
// advances the axion: Gamma_a from phi^n and the source S_a that kernel A left
// in scratch, the transport of T_a^+- by one cell (neighbouring cells' new
// values by lane shuffles) and phi^{n+1}; the chunk's lower halo row is
// advanced the same way without being stored.  The 18 per-mode factors of
// j_a are exchanged through LDS between the waves in two phases (four
// barriers per row), and each wave evaluates C_m for its own mode.  The
// factors (qds_current_rows.hpp) are those of ja_factors with the
// transport-variable form of the theta and r components.
#include "qds_current_rows.hpp"

namespace qds {
namespace cur {

constexpr int OWN = kFusedOwn;

// Output stores of the march.  In FP64 they are streaming stores, which keep
// T_a, phi and j_a out of the caches: kernel B, which runs next, measured 3%
// faster (the FP64 step 0.5-1%).  In FP32, and for the stores of kernels A
// and B, the hint was neutral or slower.
template <typename T>
__device__ __forceinline__ void sto_out(cx<T>* p, uint32_t o, cx<T> v) {
    cx<T>* q = (cx<T>*)((g_char*)(p) + o);
    if constexpr (sizeof(T) == 8) st_nt(q, v);
    else st(q, v);
}

template <typename T>
__device__ __forceinline__ cx<T> shfl_up1(cx<T> v) {
    return cx<T>{__shfl_up(v.re, 1, WAVE), __shfl_up(v.im, 1, WAVE)};
}
template <typename T>
__device__ __forceinline__ cx<T> shfl_dn1(cx<T> v) {
    return cx<T>{__shfl_down(v.re, 1, WAVE), __shfl_down(v.im, 1, WAVE)};
}

template <typename T, int M>
__device__ __forceinline__ void current_body(const AxionArgs<T>& a, int strip, int chunk, int rows) {
    const Geo& g = a.g;
    const int m = threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    const int raw = strip * OWN - 1 + lane;
    const bool inrange = raw >= 0 && raw < g.nx;
    // halo lanes wrap with periodic x and are clamped otherwise
    const int i = g.per ? ((raw % g.nx) + g.nx) % g.nx : (raw < 0 ? 0 : (raw >= g.nx ? g.nx - 1 : raw));
    const bool owner = inrange && lane >= 1 && lane <= OWN;
    const bool has1 = g.per || i + 1 < g.nx;      // column i+1 exists
    const bool live = g.per || i < g.nx - 1;
    const int i1 = (i + 1 < g.nx) ? i + 1 : (g.per ? 0 : -1);
    const int r0 = chunk * rows;
    const int r1 = min(g.nr + 1, r0 + rows);
    const T par = parity<T>(m);
    const T h = T(g.h);
    const T dr = T(g.dr);
    const T inv_dr = T(1) / dr;
    const T inv_2dr = T(0.5) * inv_dr;
    const T kap = (dr - h) / (dr + h);
    const T sj = T(a.s_j);
    const cx<T> zc = zero<T>();

    // factor exchange in two phases: j_a,x and j_a,r (12 factors), then j_a,theta (6)
    __shared__ cx<T> sm[12][M][WAVE];
    auto put = [&](int f, cx<T> v) { sm[f][m][lane] = v; };
    // out += sum over the np factor pairs from pair c0 on of +-C_m (pair sgn_pair negated)
    auto gsm = [&](int f, int k) { return sm[f][k][lane]; };
    auto convs = [&](int c0, int np, cx<T>& out, int sgn_pair) {
#pragma unroll
        for (int c = 0; c < np; ++c)
            conv_pair<T, M>(gsm, 2 * (c0 + c), 2 * (c0 + c) + 1, m, out, (c == sgn_pair) ? T(-1) : T(1));
    };

    const FacC<T> fc{m, par, tghost<T>(m), dr, inv_dr, a.bx0, a.br1, a.bt1};

    // phi^n on half row k (the exterior ghost on row nr with the open boundary)
    auto phi_row = [&](int k) {
        if (k < 0) return zc;
        if (k < g.nr) return ldo(a.phiA, eoff<T>(g, m, k, i));
        if (k == g.nr && g.open_r) return ldo(a.phiA, eoff<T>(g, m, g.nr, i));
        return zc;
    };
    // K row k < nr of the window, with the axion of that row advanced from
    // phi^n on rows k-1, k, k+1 (p_dn, p_c, p_up); store: write T_a^{n+1/2}
    // and phi^{n+1} (and on row nr - 1 the exterior ghost phi)
    auto krow = [&](int k, cx<T> p_dn, cx<T> p_c, cx<T> p_up, bool store) {
        const uint32_t o = eoff<T>(g, m, k, i);
        KRow<T> r;
        const T q = T(0.5);
        r.bxn = q * (ldo(a.A0.bx, o) + ldo(a.B0.bx, o));
        const cx<T> tpA = ldo(a.tapA, o), tmA = ldo(a.tamA, o);
        const cx<T> rpA = ldo(a.A0.trp, o), rmA = ldo(a.A0.trm, o);
        r.er0 = q * (rpA + rmA);
        r.P = q * (rpA + ldo(a.B0.trp, o));
        r.N = q * (rmA + ldo(a.B0.trm, o));
        const cx<T> Sa = ldo(a.sa, o);
        r.ph0 = p_c;
        // Gamma_a, T_a transport, phi (every lane active: DPP and shuffles)
        const T irK = T(1) / ((T(k) + T(0.5)) * dr);
        cx<T> ga = zc;
        if (live)
            ga = (inv_dr * inv_dr) * (p_up - T(2) * p_c + p_dn) + (inv_2dr * irK) * (p_up - p_dn)
                 - (T(m * m) * irK * irK + T(a.ma2)) * p_c + T(a.s_phi) * Sa;
        const cx<T> tam_b = nx1(tmA, has1);
        const cx<T> nap_b = has1 ? tpA + h * ga : zc;     // T_a^+ at column i+1
        const cx<T> nam_a = tam_b + h * ga;               // T_a^- at column i
        const cx<T> l = shfl_up1(nap_b), rr = shfl_dn1(nam_a);
        const cx<T> nap_a = (i == 0 && !g.per) ? zc : l;
        const cx<T> nam_b = has1 ? rr : zc;
        cx<T> p1 = zc;
        if (live) p1 = p_c + (h / T(4)) * (nap_a + nap_b + nam_a + nam_b);
        if (store && owner) {
            if (i1 >= 0) sto_out(a.tapB, eoff<T>(g, m, k, i1), nap_b);
            sto_out(a.tamB, o, nam_a);
            sto_out(a.phiB, o, p1);
            if (i == 0 && !g.per) sto_out(a.tapB, o, zc);
            if (k == g.nr - 1) {
                // exterior ghost phi at r_{nr+1/2}: outgoing-wave condition, two-level centring
                cx<T> Gn = p_up;
                if (g.open_r) Gn = live ? (p_c + kap * (p_up - p1)) : zc;
                sto_out(a.phiB, eoff<T>(g, m, g.nr, i), Gn);
            }
        }
        r.up = nap_a;
        r.wm = nam_a;
        r.dt0 = q * (q * (tpA + tmA) + q * (r.up + r.wm));
        r.phm = q * (r.ph0 + p1);
        return r;
    };

    // window: K row j-1, J row j; phi^n on K rows j-1 (kp.ph0) and j
    cx<T> ph_c = phi_row(r0);
    KRow<T> kp = zero_k<T>();
    if (r0 >= 1) kp = krow(r0 - 1, phi_row(r0 - 2), phi_row(r0 - 1), ph_c, false);
    JRow<T> jc = load_j(a, eoff<T>(g, m, r0, i));
    for (int j = r0; j < r1; ++j) {
        const bool calc = live && j < g.nr;
        const cx<T> ph_up = phi_row(j + 1);
        const KRow<T> kc = j < g.nr ? krow(j, kp.ph0, ph_c, ph_up, true) : zero_k<T>();
        JRow<T> jn = j + 1 <= g.nr ? load_j(a, eoff<T>(g, m, j + 1, i)) : zero_j<T>();
        const uint32_t o = eoff<T>(g, m, j, i);
        {
            // j_a,x into slots 0-5
            const NbX<T> nx = nb_x(kp, kc, jc, has1);
            if (calc) {
                cx<T> f[6];
                fac_x(fc, j, kp, kc, jc, nx, f);
#pragma unroll
                for (int q = 0; q < 6; ++q) put(q, f[q]);
            }
        }
        {
            // j_a,r into slots 6-11
            const NbR<T> nr = nb_r(kc, jc, jn, has1);
            if (calc) {
                cx<T> f[6];
                fac_r(fc, j, kc, jc, jn, nr, f);
#pragma unroll
                for (int q = 0; q < 6; ++q) put(6 + q, f[q]);
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
                sto_out(a.jax, o, sj * ox);
                if (j < g.nr) sto_out(a.jar, o, sj * orr);
            }
        }
        __syncthreads();
        {
            // j_a,theta into slots 0-5
            const NbT<T> nt = nb_t(kp, kc, jc, has1);
            if (calc) {
                cx<T> f[6];
                fac_t(fc, j, kp, kc, jc, nt, f);
#pragma unroll
                for (int q = 0; q < 6; ++q) put(q, f[q]);
            }
        }
        __syncthreads();
        {
            cx<T> ot = zc;
            if (calc) convs(0, 3, ot, 1);
            if (owner) sto_out(a.jat, o, sj * ot);
        }
        kp = kc;
        jc = jn;
        ph_c = ph_up;
        __syncthreads();
    }
}

// FP64 at three waves per SIMD (it spills a few values to scratch for it:
// measured 20% faster than two waves without spills), FP32 at five (3% faster
// than four)
template <typename T, int M>
__global__ void __launch_bounds__(WAVE * M) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 3)))
k_batch_current_march(const AxionArgs<T>* __restrict__ args, BatchList L) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int k = batch_find(L, b);
    const AxionArgs<T>& a = args[L.idx[k]];
    const int local = b - L.first[k];
    const int strips = fused_strips(a.g.nx);   // strips fastest, as kernel A
    current_body<T, M>(a, local % strips, local / strips, L.rows);
}

}  // namespace cur

int current_strips(int nx) { return fused_strips(nx); }

template <typename T>
hipError_t batch_current(const AxionArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    switch (M) {
#define QDS_BC(MM)                                                                                          \
    case MM:                                                                                                \
        hipLaunchKernelGGL((cur::k_batch_current_march<T, MM>), dim3(blocks), dim3(cur::WAVE * MM), 0, s, args, L); \
        break;
        QDS_BC(1) QDS_BC(2) QDS_BC(3) QDS_BC(4) QDS_BC(5) QDS_BC(6) QDS_BC(7) QDS_BC(8)
#undef QDS_BC
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t batch_current<double>(const AxionArgs<double>*, const BatchList&, int, int, hipStream_t);
template hipError_t batch_current<float>(const AxionArgs<float>*, const BatchList&, int, int, hipStream_t);

}  // namespace qds
