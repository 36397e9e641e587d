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
// LDS between the waves in two phases (four barriers per row), and each wave
// evaluates C_m for its own mode.  The factors (qds_current_rows.hpp) are those
// of ja_factors with the transport-variable form of the theta and r components.
#include "qds_current_rows.hpp"

namespace qds {
namespace cur {

constexpr int OWN = 63;

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

    const FacC<T> fc{m, par, dr, inv_dr, a.bx0, a.br1, a.bt1};

    // window: K row j-1, J row j
    KRow<T> kp = r0 >= 1 ? load_k(a, eoff<T>(g, m, r0 - 1, i)) : zero_k<T>();
    JRow<T> jc = load_j(a, eoff<T>(g, m, r0, i));
    for (int j = r0; j < r1; ++j) {
        const bool calc = live && j < g.nr;
        KRow<T> kc = j < g.nr ? load_k(a, eoff<T>(g, m, j, i)) : zero_k<T>();
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
                sto(a.jax, o, sj * ox);
                if (j < g.nr) sto(a.jar, o, sj * orr);
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
    const int strips = (a.g.nx + OWN - 1) / OWN;   // strips fastest, as kernel A
    current_body<T, M>(a, local % strips, local / strips, L.rows);
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
