// Per-stage kernels of one QDS step (background set, axion, regenerated set).
//
// Each kernel is a 2D stencil over (x column, radial row) that loops over the
// retained modes; a step is a short sequence of them on one stream, reading
// the old state from buffer A and writing the new one to buffer B.  These
// stages are the plain form of the step; the fused single-pass step in
// qds_fused.hip computes the same values and is checked against them.
#include "qds_stage_ops.hpp"

namespace qds {

// prescribed j_x^(0) at (x_{i+1/2}, r_j, t^n), lab column i + w
template <typename T>
__device__ __forceinline__ T drive_jx(const Drive& d, const Geo& g, int i, int j, int64_t n, int64_t w) {
    const double x = (double(i) + 0.5 + double(w)) * g.h;
    const double t = double(n) * g.h;
    const double r = double(j) * g.dr;
    const double ax = x - d.x0 - d.v * t;
    const double ar = r - d.r0;
    const double gx = exp(-ax * ax / (2.0 * d.sx * d.sx));
    const double gr = exp(-ar * ar / (2.0 * d.sr * d.sr));
    const uint64_t c = (uint64_t(n) << 32) | (uint64_t(int64_t(i) + w) << 12) | uint64_t(j);
    const double xi = normal_ctr(d.seed, c);
    return T(d.amp * gr * gx * (1.0 + d.noise * xi));
}

// total current j_x at (x_{i+1/2}, r_j, t^n) of set s: plasma + extra
template <typename T>
__device__ __forceinline__ cx<T> jx_total(const StageArgs<T>& a, int m, int j, int i) {
    const Geo& g = a.g;
    int c = i;
    if (g.per) {
        c = (i + g.nx) % g.nx;
    } else if (i < 0 || i >= g.nx - 1) {
        return zero<T>();          // outside the domain or the dead half column
    }
    cx<T> v = zero<T>();
    if (a.plasma) v = ld(a.B.jx + g.at(m, j, c));     // j_x^n, written by the longitudinal stage
    if (a.jx_add) v = v + ld(a.jx_add + g.at(m, j, c));
    if (a.drive.on && m == 0) v.re += drive_jx<T>(a.drive, g, c, j, a.n, a.w);
    // particle deposits: j_x^n as the mean of the steps ending at t^{n-1/2}, t^{n+1/2}
    if (a.pjx0) v = v + T(0.5) * ld(a.pjx0 + g.at(m, j, c));
    if (a.pjx1) v = v + T(0.5) * ld(a.pjx1 + g.at(m, j, c));
    return v;
}

// plasma j at t^{n+1/2} (written to B by the longitudinal stage), x-averaged to
// x_{i+1/2}, plus the extra current already at the source point
template <typename T>
__device__ __forceinline__ cx<T> jr_total(const StageArgs<T>& a, int m, int k, int i) {
    const Geo& g = a.g;
    cx<T> v = zero<T>();
    if (a.plasma) v = T(0.5) * (ldx(a.B.jr, g, m, k, i) + ldx(a.B.jr, g, m, k, i + 1));
    if (a.jr_add) v = v + ld(a.jr_add + g.at(m, k, i));
    if (a.pjr) v = v + T(0.5) * (ldx(a.pjr, g, m, k, i) + ldx(a.pjr, g, m, k, i + 1));
    return v;
}
template <typename T>
__device__ __forceinline__ cx<T> jt_total(const StageArgs<T>& a, int m, int j, int i) {
    const Geo& g = a.g;
    cx<T> v = zero<T>();
    if (a.plasma) v = T(0.5) * (ldx(a.B.jt, g, m, j, i) + ldx(a.B.jt, g, m, j, i + 1));
    if (a.jt_add) v = v + ld(a.jt_add + g.at(m, j, i));
    if (a.pjt) v = v + T(0.5) * (ldx(a.pjt, g, m, j, i) + ldx(a.pjt, g, m, j, i + 1));
    return v;
}

// ---------------------------------------------------------------------------
// stage 1: plasma currents and the longitudinal leapfrog E_x, B_x
// (Eqs. Ex_update, Gammax_explicit, Phix_explicit, axis_Ex, em_r_open_bx)
// one thread per (column i, row j), j = 0..nr
// ---------------------------------------------------------------------------
template <typename T>
__device__ cx<T> bx_new_at(const StageArgs<T>& a, int m, int k, int i) {
    // B_x^{n+1/2} at (x_{i+1/2}, r_{k+1/2}), k < nr
    const Geo& g = a.g;
    const T dr = T(g.dr), h = T(g.h);
    const T rk = (T(k) + T(0.5)) * dr;
    cx<T> lo0 = eth(a.A, g, m, k, i), lo1 = eth(a.A, g, m, k, i + 1);
    cx<T> hi0 = eth(a.A, g, m, k + 1, i), hi1 = eth(a.A, g, m, k + 1, i + 1);
    cx<T> eavg = T(0.25) * (lo0 + hi0 + lo1 + hi1);
    cx<T> de = (T(1) / (T(2) * dr)) * ((hi0 + hi1) - (lo0 + lo1));
    cx<T> eravg = T(0.5) * (er(a.A, g, m, k, i) + er(a.A, g, m, k, i + 1));
    cx<T> fx = -((T(1) / rk) * eavg + de) - imul(T(m) / rk, eravg);
    return ld(a.A.bx + g.at(m, k, i)) + h * fx;
}

template <typename T>
__global__ void __launch_bounds__(256) k_longitudinal(StageArgs<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j > g.nr) return;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = g.per || i < g.nx - 1;
    const T wp2h = T(a.wp2 * g.h);
    for (int m = 0; m < g.M; ++m) {
        const size_t e = g.at(m, j, i);
        // plasma response (j_x to t^n, j_r and j_theta to t^{n+1/2})
        if (a.plasma) {
            st(a.B.jx + e, ld(a.A.jx + e) + wp2h * ld(a.A.ex + e));
            if (j < g.nr) st(a.B.jr + e, ld(a.A.jr + e) + wp2h * er(a.A, g, m, j, i));
            cx<T> jt = ld(a.A.jt + e) + wp2h * eth(a.A, g, m, j, i);
            if (!g.open_r && j == g.nr) jt = zero<T>();
            st(a.B.jt + e, jt);
        }
    }
    for (int m = 0; m < g.M; ++m) {
        const size_t e = g.at(m, j, i);
        // ---- E_x at (x_{i+1/2}, r_j)
        cx<T> exn;
        if (!live || (!g.open_r && j == g.nr)) {
            exn = zero<T>();
        } else if (j == 0) {
            if (m == 0) {
                cx<T> b = T(0.5) * (bth(a.A, g, 0, 0, i) + bth(a.A, g, 0, 0, i + 1));
                cx<T> gx = (T(4) / dr) * b - jx_total(a, 0, 0, i);
                exn = ld(a.A.ex + e) + h * gx;
            } else {
                exn = zero<T>();
            }
        } else {
            const T rj = T(j) * dr;
            cx<T> lo0 = bth(a.A, g, m, j - 1, i), lo1 = bth(a.A, g, m, j - 1, i + 1);
            cx<T> hi0 = bth(a.A, g, m, j, i), hi1 = bth(a.A, g, m, j, i + 1);
            cx<T> bavg = T(0.25) * (lo0 + hi0 + lo1 + hi1);
            cx<T> db = (T(1) / (T(2) * dr)) * ((hi0 + hi1) - (lo0 + lo1));
            cx<T> bravg = T(0.5) * (brr(a.A, g, m, j, i) + brr(a.A, g, m, j, i + 1));
            cx<T> gx = (T(1) / rj) * bavg + db + imul(T(m) / rj, bravg) - jx_total(a, m, j, i);
            exn = ld(a.A.ex + e) + h * gx;
        }
        st(a.B.ex + e, exn);
        // ---- B_x at (x_{i+1/2}, r_{j+1/2}), and the exterior ghost row
        if (j < g.nr) {
            st(a.B.bx + e, live ? bx_new_at(a, m, j, i) : zero<T>());
        } else {
            cx<T> gh = zero<T>();
            if (g.open_r && live) {
                const int N = g.nr;
                const T rN = T(N) * dr;
                const T kap = (dr - h) / (dr + h), cR = T(2) * h * dr / (dr + h);
                cx<T> rx = (T(0.5) / h) * (brr(a.A, g, m, N, i + 1) - brr(a.A, g, m, N, i));
                cx<T> ea = T(0.5) * (eth(a.A, g, m, N, i) + eth(a.A, g, m, N, i + 1));
                cx<T> ra = T(0.5) * (er(a.A, g, m, N - 1, i) + er(a.A, g, m, N - 1, i + 1));
                rx = rx - (T(1) / (T(2) * rN)) * (ea + imul(T(m), ra));
                // j_theta at (x_{i+1/2}, r_nr, t^{n+1/2}): plasma part recomputed
                // here from the old state (B.jt of column i+1 may not be written yet)
                cx<T> jt = zero<T>();
                if (a.plasma) {
                    cx<T> j0 = ldx(a.A.jt, g, m, N, i) + wp2h * eth(a.A, g, m, N, i);
                    cx<T> j1 = ldx(a.A.jt, g, m, N, i + 1) + wp2h * eth(a.A, g, m, N, i + 1);
                    jt = T(0.5) * (j0 + j1);
                }
                if (a.jt_add) jt = jt + ld(a.jt_add + g.at(m, N, i));
                if (a.pjt) jt = jt + T(0.5) * (ldx(a.pjt, g, m, N, i) + ldx(a.pjt, g, m, N, i + 1));
                rx = rx - T(0.5) * jt;
                cx<T> I0 = ld(a.A.bx + g.at(m, N - 1, i));
                cx<T> I1 = bx_new_at(a, m, N - 1, i);
                cx<T> G0 = ld(a.A.bx + g.at(m, N, i));
                gh = I0 + kap * (G0 - I1) + cR * rx;
            }
            st(a.B.bx + e, gh);
        }
    }
}

// ---------------------------------------------------------------------------
// stage 2: transverse transport (Eqs. Trp/Trm/Ttp/Ttm_update, axis_Ttheta,
// em_x_open): thread (i, j) owns the source at x_{i+1/2} and writes the right
// movers at column i+1 and the left movers at column i
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_transverse(StageArgs<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j > g.nr) return;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = g.per || i < g.nx - 1;
    const int ir = g.per ? (i + 1) % g.nx : i + 1;     // destination of right movers
    for (int m = 0; m < g.M; ++m) {
        // ---- T_r on half row j
        if (j < g.nr) {
            cx<T> sp = zero<T>(), sm = zero<T>();
            if (live) {
                const T rk = (T(j) + T(0.5)) * dr;
                cx<T> gr = -imul(T(m) / rk, ld(a.B.bx + g.at(m, j, i))) - jr_total(a, m, j, i);
                cx<T> pr = (T(1) / dr) * (ld(a.B.ex + g.at(m, j + 1, i)) - ld(a.B.ex + g.at(m, j, i)));
                sp = h * (gr + pr);
                sm = h * (gr - pr);
            }
            if (ir < g.nx) st(a.B.trp + g.at(m, j, ir), ldx(a.A.trp, g, m, j, i) + sp);
            st(a.B.trm + g.at(m, j, i), ldx(a.A.trm, g, m, j, i + 1) + sm);
            if (i == 0 && !g.per) st(a.B.trp + g.at(m, j, 0), zero<T>());
        }
        // ---- T_theta on integer row j
        bool zero_row = (!g.open_r && j == g.nr) || (j == 0 && m != 1);
        cx<T> sp = zero<T>(), sm = zero<T>();
        if (live && !zero_row) {
            cx<T> gt, pt;
            if (j == 0) {
                gt = -(T(2) / dr) * ld(a.B.bx + g.at(1, 0, i)) - jt_total(a, 1, 0, i);
                pt = imul(T(1) / dr, ld(a.B.ex + g.at(1, 1, i)));
            } else {
                const T rj = T(j) * dr;
                gt = -(T(1) / dr) * (ld(a.B.bx + g.at(m, j, i)) - ld(a.B.bx + g.at(m, j - 1, i)))
                     - jt_total(a, m, j, i);
                pt = imul(T(m) / rj, ld(a.B.ex + g.at(m, j, i)));
            }
            sp = h * (gt + pt);
            sm = h * (gt - pt);
        }
        if (zero_row) {
            st(a.B.ttp + g.at(m, j, i), zero<T>());
            if (ir < g.nx) st(a.B.ttm + g.at(m, j, ir), zero<T>());
        } else {
            st(a.B.ttp + g.at(m, j, i), ldx(a.A.ttp, g, m, j, i + 1) + sp);
            if (ir < g.nx) st(a.B.ttm + g.at(m, j, ir), ldx(a.A.ttm, g, m, j, i) + sm);
        }
        if (i == 0 && !g.per) st(a.B.ttm + g.at(m, j, 0), zero<T>());
    }
}

// ---------------------------------------------------------------------------
// stage 3: exterior ghost B_theta at r_{nr+1/2} (Eq. em_r_open_bt), one thread
// per column
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_ghost_bth(StageArgs<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nx) return;
    const int N = g.nr;
    const T h = T(g.h), dr = T(g.dr);
    const T rN = T(N) * dr;
    const T kap = (dr - h) / (dr + h), cR = T(2) * h * dr / (dr + h);
    for (int m = 0; m < g.M; ++m) {
        cx<T> out = zero<T>();
        if (g.open_r) {
            cx<T> I0 = bth(a.A, g, m, N - 1, i);
            cx<T> I1 = T(0.5) * (ld(a.B.trp + g.at(m, N - 1, i)) - ld(a.B.trm + g.at(m, N - 1, i)));
            cx<T> G0 = ld(a.A.trp + g.at(m, N, i));
            cx<T> dxer = (T(1) / (T(2) * h)) * (er(a.A, g, m, N - 1, i + 1) - er(a.A, g, m, N - 1, i - 1));
            cx<T> jxi = T(0.5) * (jx_total(a, m, N, i) + jx_total(a, m, N, i - 1));
            cx<T> rt = -T(0.5) * dxer - (T(1) / (T(2) * rN)) * (T(0.5) * (I0 + G0) + imul(T(m), brr(a.A, g, m, N, i)))
                       + T(0.5) * jxi;
            out = I0 + kap * (G0 - I1) + cR * rt;
        }
        st(a.B.trp + g.at(m, N, i), out);
        st(a.B.trm + g.at(m, N, i), zero<T>());
    }
}

// ---------------------------------------------------------------------------
// theta-grid evaluation of the mode products (Sec. 3.3: transform the factors
// to a discrete theta grid, multiply pointwise, transform back), in place of
// the direct convolution C_m.  A product of two fields with modes below M
// has modes up to 2M - 2; on N equispaced points the coefficient of mode
// m < M picks up the alias N - m of the product, so N = 3M - 2 points are the
// fewest that leave modes 0..M-1 exact.  At these N a table-driven DFT (the
// table in LDS, filled once per block) does the transforms.  Real samples see
// only Re A^(0); the literal convolution's mode 0 uses the complex product
// A^(0) B^(0) (while its modes m >= 1 use Re A^(0), Re B^(0) like the grid),
// so the difference A^(0) B^(0) - Re A^(0) Re B^(0) is added to mode 0.
// ---------------------------------------------------------------------------
template <int M>
__host__ __device__ constexpr int theta_points() { return 3 * M - 2; }

template <int M>
__device__ void theta_table(double* tc, double* ts) {
    constexpr int N = theta_points<M>();
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
    for (int q = t; q < M * N; q += blockDim.x * blockDim.y) {
        const int m = q / N, k = q % N;
        double sn, cs;
        sincospi(2.0 * double((m * k) % N) / double(N), &sn, &cs);
        tc[q] = cs;
        ts[q] = sn;
    }
    __syncthreads();
}

// Re sum_m A^(m) e^{-i m theta_k}
template <typename T, int M>
__device__ __forceinline__ T theta_eval(const cx<T>* A, const double* tc, const double* ts, int k) {
    constexpr int N = theta_points<M>();
    T v = A[0].re;
#pragma unroll
    for (int m = 1; m < M; ++m) v += A[m].re * T(tc[m * N + k]) + A[m].im * T(ts[m * N + k]);
    return v;
}

// out^(m) += (1 or 2)/N p_k e^{i m theta_k}
template <typename T, int M>
__device__ __forceinline__ void theta_project(T p, cx<T>* out, const double* tc, const double* ts, int k) {
    constexpr int N = theta_points<M>();
    const T w0 = T(1.0 / N), w = T(2.0 / N);
    out[0].re += w0 * p;
#pragma unroll
    for (int m = 1; m < M; ++m) {
        out[m].re += (w * p) * T(tc[m * N + k]);
        out[m].im += (w * p) * T(ts[m * N + k]);
    }
}

template <typename T>
__device__ __forceinline__ void theta_mode0_fix(cx<T> a, cx<T> b, T sign, cx<T>& out0) {
    out0 = out0 + sign * cx<T>{-a.im * b.im, a.re * b.im + a.im * b.re};
}

// out += s0 C{A0, B0} + s1 C{A1, B1} + s2 C{A2, B2} on the theta grid
template <typename T, int M>
__device__ __forceinline__ void theta_acc3(const cx<T>* A0, const cx<T>* B0, T s0, const cx<T>* A1, const cx<T>* B1,
                                           T s1, const cx<T>* A2, const cx<T>* B2, T s2, cx<T>* out,
                                           const double* tc, const double* ts) {
    constexpr int N = theta_points<M>();
#pragma unroll 2
    for (int k = 0; k < N; ++k) {
        const T p = s0 * theta_eval<T, M>(A0, tc, ts, k) * theta_eval<T, M>(B0, tc, ts, k) +
                    s1 * theta_eval<T, M>(A1, tc, ts, k) * theta_eval<T, M>(B1, tc, ts, k) +
                    s2 * theta_eval<T, M>(A2, tc, ts, k) * theta_eval<T, M>(B2, tc, ts, k);
        theta_project<T, M>(p, out, tc, ts, k);
    }
    theta_mode0_fix(A0[0], B0[0], s0, out[0]);
    theta_mode0_fix(A1[0], B1[0], s1, out[0]);
    theta_mode0_fix(A2[0], B2[0], s2, out[0]);
}

// ---------------------------------------------------------------------------
// stage 4: axion source S_a, Gamma_a and the T_a shift (Eqs.
// mode_convolution, Ta_plus_update, Ta_minus_update, axion_x_open)
// ---------------------------------------------------------------------------
template <typename T, int M, bool THETA>
__global__ void __launch_bounds__(256) k_axion_ta(AxionArgs<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y * blockDim.y + threadIdx.y;
    __shared__ double tc[THETA ? M * theta_points<M>() : 1], ts[THETA ? M * theta_points<M>() : 1];
    if constexpr (THETA) theta_table<M>(tc, ts);
    if (i >= g.nx || k >= g.nr) return;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = g.per || i < g.nx - 1;
    const int ir = g.per ? (i + 1) % g.nx : i + 1;
    cx<T> S[M];
#pragma unroll
    for (int m = 0; m < M; ++m) S[m] = zero<T>();
    if (live) {
        // transverse part in transport variables (exact rewrite of
        // C{E_r, B_r} + C{E_th, B_th}, free of the cancellation between the
        // two products for co-propagating waves):
        //   1/2 C{T_r^+ + b_th, T_th^+ + b_r} - 1/2 C{T_r^- - b_th, T_th^- - b_r}
        cx<T> Ex[M], Bx[M], Pp[M], Qp[M], Pm[M], Qm[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            Pp[m] = T(0.25) * (ldx(a.A0.trp, g, m, k, i) + ldx(a.A0.trp, g, m, k, i + 1));
            Pm[m] = T(-0.25) * (ldx(a.A0.trm, g, m, k, i) + ldx(a.A0.trm, g, m, k, i + 1));
            Qp[m] = T(0.25) * (ldx(a.A0.ttp, g, m, k, i) + ldx(a.A0.ttp, g, m, k + 1, i) + ldx(a.A0.ttp, g, m, k, i + 1) +
                               ldx(a.A0.ttp, g, m, k + 1, i + 1));
            Qm[m] = T(0.25) * (ldx(a.A0.ttm, g, m, k, i) + ldx(a.A0.ttm, g, m, k + 1, i) + ldx(a.A0.ttm, g, m, k, i + 1) +
                               ldx(a.A0.ttm, g, m, k + 1, i + 1));
            cx<T> e0 = T(0.5) * (ld(a.A0.ex + g.at(m, k, i)) + ld(a.B0.ex + g.at(m, k, i)));
            cx<T> e1 = T(0.5) * (ld(a.A0.ex + g.at(m, k + 1, i)) + ld(a.B0.ex + g.at(m, k + 1, i)));
            Ex[m] = T(0.5) * (e0 + e1);
            Bx[m] = T(0.5) * (ld(a.A0.bx + g.at(m, k, i)) + ld(a.B0.bx + g.at(m, k, i)));
        }
        Bx[0] = Bx[0] + a.bx0;
        if (M > 1) {
            Pp[1] = Pp[1] + T(0.5) * a.bt1;
            Pm[1] = Pm[1] + T(0.5) * a.bt1;
            Qp[1] = Qp[1] + a.br1;
            Qm[1] = Qm[1] - a.br1;
        }
        if constexpr (THETA) {
            theta_acc3<T, M>(Ex, Bx, T(1), Pp, Qp, T(1), Pm, Qm, T(1), S, tc, ts);
        } else {
            conv_acc<T, M>(Ex, Bx, T(1), S);
            conv_acc<T, M>(Pp, Qp, T(1), S);
            conv_acc<T, M>(Pm, Qm, T(1), S);
        }
    }
    const T rk = (T(k) + T(0.5)) * dr;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        cx<T> ga = zero<T>();
        if (live) {
            cx<T> p = ld(a.phiA + g.at(m, k, i));
            cx<T> up = (k + 1 < g.nr) ? ld(a.phiA + g.at(m, k + 1, i))
                                      : (g.open_r ? ld(a.phiA + g.at(m, g.nr, i)) : zero<T>());
            cx<T> dn = (k > 0) ? ld(a.phiA + g.at(m, k - 1, i)) : zero<T>();
            ga = (T(1) / (dr * dr)) * (up - T(2) * p + dn) + (T(1) / (T(2) * dr * rk)) * (up - dn)
                 - (T(m * m) / (rk * rk) + T(a.ma2)) * p + T(a.s_phi) * S[m];
        }
        if (ir < g.nx) st(a.tapB + g.at(m, k, ir), ldx(a.tapA, g, m, k, i) + h * ga);
        st(a.tamB + g.at(m, k, i), ldx(a.tamA, g, m, k, i + 1) + h * ga);
        if (i == 0 && !g.per) st(a.tapB + g.at(m, k, 0), zero<T>());
    }
}

// stage 5: phi^{n+1} from T_a^{n+1/2} (Eq. phi_update) and the exterior ghost
template <typename T>
__global__ void __launch_bounds__(256) k_axion_phi(AxionArgs<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || k >= g.nr) return;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = g.per || i < g.nx - 1;
    const T kap = (dr - h) / (dr + h);
    for (int m = 0; m < g.M; ++m) {
        cx<T> p = zero<T>();
        if (live) {
            cx<T> s = ldx(a.tapB, g, m, k, i) + ldx(a.tapB, g, m, k, i + 1) + ldx(a.tamB, g, m, k, i) +
                      ldx(a.tamB, g, m, k, i + 1);
            p = ld(a.phiA + g.at(m, k, i)) + (h / T(4)) * s;
        }
        st(a.phiB + g.at(m, k, i), p);
        if (k == g.nr - 1) {
            cx<T> G = ld(a.phiA + g.at(m, g.nr, i));
            cx<T> Gn = G;
            if (g.open_r) Gn = live ? (ld(a.phiA + g.at(m, k, i)) + kap * (G - p)) : zero<T>();
            st(a.phiB + g.at(m, g.nr, i), Gn);
        }
    }
}

// ---------------------------------------------------------------------------
// stage 6: axion current j_a for the regenerated set (Eqs. jax_mode,
// jar_mode, jat_mode) at the source points x_{i+1/2}: j_a,x at (r_j, t^n),
// j_a,r at (r_{j+1/2}, t^{n+1/2}), j_a,theta at (r_j, t^{n+1/2})
// ---------------------------------------------------------------------------
// One component of the axion current (PART 0: j_a,x, 1: j_a,theta, 2: j_a,r):
// out += C{f0, f1} - C{f2, f3} + C{f4, f5} of that component's factors.
template <typename T, int M, bool THETA, int PART>
__device__ __forceinline__ void comp_products(const AxionArgs<T>& a, int i, int j, cx<T>* out, const double* tc,
                                              const double* ts) {
    cx<T> F[6][M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        cx<T> f[18];
        ja_factors<T, true, PART>(a, m, i, j, f);
#pragma unroll
        for (int q = 0; q < 6; ++q) F[q][m] = f[6 * PART + q];
    }
    if constexpr (THETA) {
        theta_acc3<T, M>(F[0], F[1], T(1), F[2], F[3], T(-1), F[4], F[5], T(1), out, tc, ts);
    } else {
        conv_acc<T, M>(F[0], F[1], T(1), out);
        conv_acc<T, M>(F[2], F[3], T(-1), out);
        conv_acc<T, M>(F[4], F[5], T(1), out);
    }
}

template <typename T, int M, bool THETA>
__global__ void __launch_bounds__(256) k_axion_current(AxionArgs<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    __shared__ double tc[THETA ? M * theta_points<M>() : 1], ts[THETA ? M * theta_points<M>() : 1];
    if constexpr (THETA) theta_table<M>(tc, ts);
    if (i >= g.nx || j > g.nr) return;
    const bool live = g.per || i < g.nx - 1;
    cx<T> jx[M], jr[M], jt[M];
#pragma unroll
    for (int m = 0; m < M; ++m) jx[m] = jr[m] = jt[m] = zero<T>();
    if (live && j < g.nr) {
        if constexpr (THETA) {
            // one component at a time (its six factor arrays): the theta-grid
            // products of the many-mode cases then stay close to the register
            // file (the direct convolution spills more this way and keeps all
            // 18 factor arrays)
            comp_products<T, M, THETA, 0>(a, i, j, jx, tc, ts);
            comp_products<T, M, THETA, 1>(a, i, j, jt, tc, ts);
            comp_products<T, M, THETA, 2>(a, i, j, jr, tc, ts);
        } else {
            cx<T> F[18][M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                cx<T> f[18];
                ja_factors<T, true>(a, m, i, j, f);
#pragma unroll
                for (int q = 0; q < 18; ++q) F[q][m] = f[q];
            }
            conv_acc<T, M>(F[0], F[1], T(1), jx);
            conv_acc<T, M>(F[2], F[3], T(-1), jx);
            conv_acc<T, M>(F[4], F[5], T(1), jx);
            conv_acc<T, M>(F[6], F[7], T(1), jt);
            conv_acc<T, M>(F[8], F[9], T(-1), jt);
            conv_acc<T, M>(F[10], F[11], T(1), jt);
            conv_acc<T, M>(F[12], F[13], T(1), jr);
            conv_acc<T, M>(F[14], F[15], T(-1), jr);
            conv_acc<T, M>(F[16], F[17], T(1), jr);
        }
    }
    const T sj = T(a.s_j);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        st(a.jax + g.at(m, j, i), sj * jx[m]);
        st(a.jat + g.at(m, j, i), sj * jt[m]);
        if (j < g.nr) st(a.jar + g.at(m, j, i), sj * jr[m]);
    }
}


// ---------------------------------------------------------------------------
// particle currents at the source points (read by the fused background march
// as its extra currents; the staged stages form the same sums in place)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_particle_sources(const cx<T>* __restrict__ pjx0, const cx<T>* __restrict__ pjx1,
                                                          const cx<T>* __restrict__ pjr, const cx<T>* __restrict__ pjt,
                                                          Geo g, cx<T>* __restrict__ out, size_t plane) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;                // 0..nr
    const int m = blockIdx.z;
    if (i >= g.nx) return;
    const size_t e = g.at(m, row, i);
    cx<T> jx = zero<T>();
    if (pjx0) jx = jx + T(0.5) * ld(pjx0 + e);
    jx = jx + T(0.5) * ld(pjx1 + e);
    const cx<T> jr = row < g.nr ? T(0.5) * (ldx(pjr, g, m, row, i) + ldx(pjr, g, m, row, i + 1)) : zero<T>();
    const cx<T> jt = T(0.5) * (ldx(pjt, g, m, row, i) + ldx(pjt, g, m, row, i + 1));
    st(out + e, jx);
    st(out + plane + e, jr);
    st(out + 2 * plane + e, jt);
}

template <typename T>
hipError_t particle_sources(const cx<T>* pjx0, const cx<T>* pjx1, const cx<T>* pjr, const cx<T>* pjt, const Geo& g,
                            cx<T>* out, size_t plane_elems, hipStream_t s) {
    hipLaunchKernelGGL((k_particle_sources<T>), dim3((g.nx + 255) / 256, g.nr + 1, g.M), dim3(256), 0, s, pjx0, pjx1,
                       pjr, pjt, g, out, plane_elems);
    return hipGetLastError();
}
template hipError_t particle_sources<double>(const cx<double>*, const cx<double>*, const cx<double>*, const cx<double>*,
                                             const Geo&, cx<double>*, size_t, hipStream_t);
template hipError_t particle_sources<float>(const cx<float>*, const cx<float>*, const cx<float>*, const cx<float>*,
                                            const Geo&, cx<float>*, size_t, hipStream_t);

// ---------------------------------------------------------------------------
// moving window: copy every plane shifted left by one column, zero the last
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_window_shift(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, Geo g, int nplanes) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;           // over planes * modes * (nr+1)
    if (i >= g.nx) return;
    const size_t base = size_t(row) * g.ld;
    cx<T> v = (i + 1 < g.nx) ? ld(src + base + i + 1) : zero<T>();
    st(dst + base + i, v);
}

// ---------------------------------------------------------------------------
// pulse loading: add a forward pulse to set 0 (the mode content of a linear,
// radial or azimuthal polarisation with B = x_hat x E)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_add_pulse(SetPtr<T> s, Geo g, int pol, const double* fK, const double* fJ, const double* fG) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= g.nx || j > g.nr) return;
    // (E_r, E_theta, B_r, B_theta) of mode ``md`` per unit real field f
    int md;
    cx<T> er, et, br, bt;
    const cx<T> one = {T(1), T(0)}, ii = {T(0), T(1)};
    switch (pol) {
        case 'y': md = 1; er = one; et = -ii; br = ii; bt = one; break;
        case 'z': md = 1; er = ii; et = one; br = -one; bt = ii; break;
        case 'r': md = 0; er = one; et = zero<T>(); br = zero<T>(); bt = one; break;
        default:  md = 0; er = zero<T>(); et = one; br = -one; bt = zero<T>(); break;
    }
    if (md >= g.M) return;
    if (j < g.nr) {
        const T f = T(fK[size_t(j) * g.nx + i]);
        const size_t e = g.at(md, j, i);
        st(s.trp + e, ld(s.trp + e) + f * (er + bt));
        st(s.trm + e, ld(s.trm + e) + f * (er - bt));
    } else if (g.open_r) {
        const size_t e = g.at(md, g.nr, i);
        st(s.trp + e, ld(s.trp + e) + T(fG[i]) * bt);
    }
    const bool axis_zero = (j == 0 && md != 1) || (!g.open_r && j == g.nr);
    if (!axis_zero) {
        const T f = T(fJ[size_t(j) * g.nx + i]);
        const size_t e = g.at(md, j, i);
        st(s.ttp + e, ld(s.ttp + e) + f * (et + br));
        st(s.ttm + e, ld(s.ttm + e) + f * (et - br));
    }
}

// ---------------------------------------------------------------------------
// host-side launch sequence of the staged step
// ---------------------------------------------------------------------------
template <typename T, int M>
static void launch_axion(AxionArgs<T>& ax, bool arem, bool theta, hipStream_t s) {
    const Geo& g = ax.g;
    dim3 blk(64, 4);
    dim3 grdK((g.nx + 63) / 64, (g.nr + 3) / 4);
    dim3 grdJ((g.nx + 63) / 64, (g.nr + 1 + 3) / 4);
    if (theta) hipLaunchKernelGGL((k_axion_ta<T, M, true>), grdK, blk, 0, s, ax);
    else hipLaunchKernelGGL((k_axion_ta<T, M, false>), grdK, blk, 0, s, ax);
    hipLaunchKernelGGL(k_axion_phi<T>, grdK, blk, 0, s, ax);
    if (arem) {
        if (theta) hipLaunchKernelGGL((k_axion_current<T, M, true>), grdJ, blk, 0, s, ax);
        else hipLaunchKernelGGL((k_axion_current<T, M, false>), grdJ, blk, 0, s, ax);
    }
}

template <typename T>
hipError_t staged_step(const StepPlan<T>& p, hipStream_t s) {
    const Geo& g = p.g;
    dim3 blk(64, 4);
    dim3 grdJ((g.nx + 63) / 64, (g.nr + 1 + 3) / 4);
    // ---- background set
    StageArgs<T> a0 = p.set_args(0);
    hipLaunchKernelGGL(k_longitudinal<T>, grdJ, blk, 0, s, a0);
    hipLaunchKernelGGL(k_transverse<T>, grdJ, blk, 0, s, a0);
    hipLaunchKernelGGL(k_ghost_bth<T>, dim3((g.nx + 255) / 256), dim3(256), 0, s, a0);
    // ---- axion
    if (p.axion) {
        AxionArgs<T> ax = p.axion_args();
        switch (g.M) {
#define QDS_AX_CASE(MM) case MM: launch_axion<T, MM>(ax, p.arem, p.theta != 0, s); break;
            QDS_AX_CASE(1) QDS_AX_CASE(2) QDS_AX_CASE(3) QDS_AX_CASE(4)
            QDS_AX_CASE(5) QDS_AX_CASE(6) QDS_AX_CASE(7) QDS_AX_CASE(8)
#undef QDS_AX_CASE
            default: return hipErrorInvalidValue;
        }
        if (p.arem) {
            StageArgs<T> a1 = p.set_args(1);
            hipLaunchKernelGGL(k_longitudinal<T>, grdJ, blk, 0, s, a1);
            hipLaunchKernelGGL(k_transverse<T>, grdJ, blk, 0, s, a1);
            hipLaunchKernelGGL(k_ghost_bth<T>, dim3((g.nx + 255) / 256), dim3(256), 0, s, a1);
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t window_shift(const cx<T>* src, cx<T>* dst, const Geo& g, int nplanes, hipStream_t s) {
    dim3 grd((g.nx + 255) / 256, nplanes * g.M * (g.nr + 1));
    hipLaunchKernelGGL(k_window_shift<T>, grd, dim3(256), 0, s, src, dst, g, nplanes);
    return hipGetLastError();
}

template <typename T>
hipError_t add_pulse(SetPtr<T> s0, const Geo& g, int pol, const double* fK, const double* fJ, const double* fG,
                     hipStream_t s) {
    dim3 grd((g.nx + 255) / 256, g.nr + 1);
    hipLaunchKernelGGL(k_add_pulse<T>, grd, dim3(256), 0, s, s0, g, pol, fK, fJ, fG);
    return hipGetLastError();
}

template hipError_t staged_step<double>(const StepPlan<double>&, hipStream_t);
template hipError_t staged_step<float>(const StepPlan<float>&, hipStream_t);
template hipError_t window_shift<double>(const cx<double>*, cx<double>*, const Geo&, int, hipStream_t);
template hipError_t window_shift<float>(const cx<float>*, cx<float>*, const Geo&, int, hipStream_t);
template hipError_t add_pulse<double>(SetPtr<double>, const Geo&, int, const double*, const double*, const double*, hipStream_t);
template hipError_t add_pulse<float>(SetPtr<float>, const Geo&, int, const double*, const double*, const double*, hipStream_t);

}  // namespace qds
