// Particle side of the cylindrical PIC coupling (Sec. 3.1), qds_particles_step
// of include/qds.h: gather of the QDS fields at the particles (Eq.
// particle_field_gather), relativistic Boris push (Eqs. boris_parameters,
// boris_update) and the charge-conserving modal deposition of the step's
// current (Eqs. particle_deposition_path .. face_current_r).
//
// One thread per particle.  The triangular particle shape gives three
// quadratic-spline weights per direction on each grid; weights that fall on a
// row below the axis are reflected onto the mirror row (r_{-1} -> r_1,
// r_{-1/2} -> r_{1/2}).  The QDS magnetic fields are first averaged along x
// onto the positions of the standard staggered interpolation (B_x to x_i,
// B_r and B_theta to x_{i+1/2}).  The transverse fields come from T^n; E_x
// and B_x are extrapolated to t^n from t^{n-1/2} and t^{n-3/2} when the
// previous level is given.  The deposit spans the old and new shapes in a
// 4 x 4 window of cells: net currents I_x, I_r per mode with the analytic
// trajectory averages of C_m (series below |m dtheta| = 0.5), face currents
// by cumulative sums from the left face and from the axis, and the angular
// current from the path's angular displacement, so that the discrete
// continuity equation holds per mode.  Currents are added with atomics.
#include <math.h>

#include "qds_ctx.hpp"

using namespace qdsi;

namespace qds {
namespace pic {

template <typename T>
struct PartArgs {
    Geo g;
    const cx<T>* trp; const cx<T>* trm; const cx<T>* ttp; const cx<T>* ttm;   // T^n of set 0
    const cx<T>* ex; const cx<T>* bx;       // t^{n-1/2}
    const cx<T>* exq; const cx<T>* bxq;     // t^{n-3/2}, or null
    double* x; double* y; double* z;
    double* ux; double* uy; double* uz;
    const double* q;
    double charge, qm;
    int64_t count;
    cx<T>* jx; cx<T>* jr; cx<T>* jt;
    unsigned long long* skipped;
};

constexpr double kPi = 3.141592653589793;

// quadratic-spline weights around the nearest node of coordinate u (in cells)
__device__ __forceinline__ int spline3(double u, double* w) {
    const int k0 = int(floor(u + 0.5));
    const double t = u - k0;
    w[0] = 0.5 * (0.5 - t) * (0.5 - t);
    w[1] = 0.75 - t * t;
    w[2] = 0.5 * (0.5 + t) * (0.5 + t);
    return k0;
}

// row of an integer (half = false) or half (half = true) radial node, reflected at the axis
__device__ __forceinline__ int fold_row(int k, bool half) { return k >= 0 ? k : (half ? -k - 1 : -k); }

template <typename T, int M>
__device__ __forceinline__ double modal(const cx<T>* P, const Geo& g, int row, int col, const double* cm,
                                        const double* sm) {
    // Re sum_m F^(m) e^{-i m theta}
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const cx<T> f = ld(P + g.at(m, row, col));
        v += double(f.re) * cm[m] + double(f.im) * sm[m];
    }
    return v;
}

// E_k(phi) = int_0^1 xi^k e^{i phi xi} dxi, k = 0, 1, 2
__device__ __forceinline__ void moments(double phi, cx<double>* E) {
    if (fabs(phi) < 0.5) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cx<double> term{1.0, 0.0}, acc{0.0, 0.0};
            for (int n = 0; n < 16; ++n) {
                acc = acc + (1.0 / double(n + k + 1)) * term;
                term = (phi / double(n + 1)) * cx<double>{-term.im, term.re};   // term *= i phi / (n + 1)
            }
            E[k] = acc;
        }
        return;
    }
    double s, c;
    sincos(phi, &s, &c);
    // 1 / (i phi) = -i / phi
    const double ip = 1.0 / phi;
    auto div_iphi = [&](cx<double> a) { return cx<double>{a.im * ip, -a.re * ip}; };
    const cx<double> e{c, s};
    E[0] = div_iphi(cx<double>{c - 1.0, s});
    E[1] = div_iphi(e - E[0]);
    E[2] = div_iphi(e - 2.0 * E[1]);
}

// Cells of the LDS deposit tile of a workgroup (three planes of one mode):
// 48 KiB.
template <typename T>
constexpr int kTileCells = 49152 / (3 * int(sizeof(cx<T>)));

// The deposit's outer loops stay rolled: 202 VGPRs in FP64, two waves per
// SIMD without spills (fully unrolled, the kernel held 256 VGPRs and ~50
// AGPRs, one wave per SIMD, or spilled ~100 registers at two).  On 983,040
// particles at 4096 x 256 x 3 sorted in 8 x 16 tiles: 0.66 ms in FP64 against
// 0.85 unrolled (three waves, spilling 48 registers: 0.95), 0.70 in FP32 at
// three waves (33 spilled) against 0.72 at two and 0.81 unrolled.
template <typename T, int M>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2)))
k_particle_step(PartArgs<T> a) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const Geo& g = a.g;
    const double h = g.h, dr = g.dr, dt = g.h;
    // what the deposit needs from the push (set by prep for an active particle)
    int ib = 0, jb = 0;
    double gx[4] = {0, 0, 0, 0}, hx[4] = {0, 0, 0, 0}, gr[4] = {0, 0, 0, 0}, hr[4] = {0, 0, 0, 0};
    double th0 = 0.0, dth = 0.0, qdt = 0.0, kth = 0.0, ax_[4], ar_[4];
    // gather and push of particle p; false when it is outside (or beyond the count)
    auto prep = [&]() -> bool {
        if (p >= a.count) return false;
        const double x0 = a.x[p], y0 = a.y[p], z0 = a.z[p];
        const double r0 = sqrt(y0 * y0 + z0 * z0);
        const double sx0 = x0 / h, sr0 = r0 / dr;
        // every stencil row and column of the gather and deposit inside the grid
        auto inside = [&](double sx, double sr) { return sx >= 2.0 && sx <= double(g.nx) - 3.0 && sr <= double(g.nr) - 2.0; };
        if (!inside(sx0, sr0)) {
            if (a.skipped) atomicAdd(a.skipped, 1ull);
            return false;
        }
        th0 = atan2(z0, y0);
        double cm[M], sm[M];
#pragma unroll
        for (int m = 0; m < M; ++m) sincos(m * th0, &sm[m], &cm[m]);

        // ---- gather
        double wxi[3], wxh[3], wrj[3], wrk[3];
        const int ci = spline3(sx0, wxi), ch = spline3(sx0 - 0.5, wxh);
        const int rj = spline3(sr0, wrj), rk = spline3(sr0 - 0.5, wrk);
        double Ex = 0, Er = 0, Et = 0, Bx = 0, Br = 0, Bt = 0;
        const bool xq = a.exq != nullptr;
        // both stencil loops stay rolled (the weights are picked by selects) so
        // that only one point's loads are in flight per iteration
        auto pick = [](const double* w, int k) { return k == 0 ? w[0] : (k == 1 ? w[1] : w[2]); };
#pragma unroll 1
        for (int q = 0; q < 9; ++q) {
            const int u = q / 3, v = q % 3;
            {
                const int J = fold_row(rj - 1 + v, false), K = fold_row(rk - 1 + v, true);
                const int cI = ci - 1 + u, cH = ch - 1 + u;
                const double wxi_u = pick(wxi, u), wxh_u = pick(wxh, u), wrj_v = pick(wrj, v), wrk_v = pick(wrk, v);
                // E_x at (x_{i+1/2}, r_j), extrapolated to t^n
                double ex = modal<T, M>(a.ex, g, J, cH, cm, sm);
                if (xq) ex = 1.5 * ex - 0.5 * modal<T, M>(a.exq, g, J, cH, cm, sm);
                Ex += wxh_u * wrj_v * ex;
                // E_r, B_theta on (x, r_{j+1/2}) from T_r; E_theta, B_r on (x, r_j) from T_theta
                const double tpK = modal<T, M>(a.trp, g, K, cI, cm, sm), tmK = modal<T, M>(a.trm, g, K, cI, cm, sm);
                Er += wxi_u * wrk_v * 0.5 * (tpK + tmK);
                const double tpJ = modal<T, M>(a.ttp, g, J, cI, cm, sm), tmJ = modal<T, M>(a.ttm, g, J, cI, cm, sm);
                Et += wxi_u * wrj_v * 0.5 * (tpJ + tmJ);
                // B_x averaged from x_{i-1/2}, x_{i+1/2} to x_i
                double bl = modal<T, M>(a.bx, g, K, cI - 1, cm, sm), br_ = modal<T, M>(a.bx, g, K, cI, cm, sm);
                if (xq) {
                    bl = 1.5 * bl - 0.5 * modal<T, M>(a.bxq, g, K, cI - 1, cm, sm);
                    br_ = 1.5 * br_ - 0.5 * modal<T, M>(a.bxq, g, K, cI, cm, sm);
                }
                Bx += wxi_u * wrk_v * 0.5 * (bl + br_);
                // B_r and B_theta averaged from x_i, x_{i+1} to x_{i+1/2}
                const double r1 = 0.5 * (modal<T, M>(a.ttp, g, J, cH, cm, sm) - modal<T, M>(a.ttm, g, J, cH, cm, sm));
                const double r2 =
                    0.5 * (modal<T, M>(a.ttp, g, J, cH + 1, cm, sm) - modal<T, M>(a.ttm, g, J, cH + 1, cm, sm));
                Br += wxh_u * wrj_v * 0.5 * (r1 + r2);
                const double t1 = 0.5 * (modal<T, M>(a.trp, g, K, cH, cm, sm) - modal<T, M>(a.trm, g, K, cH, cm, sm));
                const double t2 =
                    0.5 * (modal<T, M>(a.trp, g, K, cH + 1, cm, sm) - modal<T, M>(a.trm, g, K, cH + 1, cm, sm));
                Bt += wxh_u * wrk_v * 0.5 * (t1 + t2);
            }
        }
        // Cartesian components
        const double c0 = r0 > 0.0 ? y0 / r0 : 1.0, s0 = r0 > 0.0 ? z0 / r0 : 0.0;
        const double E[3] = {Ex, Er * c0 - Et * s0, Er * s0 + Et * c0};
        const double B[3] = {Bx, Br * c0 - Bt * s0, Br * s0 + Bt * c0};

        // ---- Boris
        const double kq = 0.5 * a.qm * dt;
        double um[3] = {a.ux[p] + kq * E[0], a.uy[p] + kq * E[1], a.uz[p] + kq * E[2]};
        const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
        const double tv[3] = {kq * B[0] / gm, kq * B[1] / gm, kq * B[2] / gm};
        const double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
        const double sv[3] = {2.0 * tv[0] / (1.0 + t2), 2.0 * tv[1] / (1.0 + t2), 2.0 * tv[2] / (1.0 + t2)};
        const double up[3] = {um[0] + (um[1] * tv[2] - um[2] * tv[1]), um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                              um[2] + (um[0] * tv[1] - um[1] * tv[0])};
        const double un[3] = {um[0] + (up[1] * sv[2] - up[2] * sv[1]) + kq * E[0],
                              um[1] + (up[2] * sv[0] - up[0] * sv[2]) + kq * E[1],
                              um[2] + (up[0] * sv[1] - up[1] * sv[0]) + kq * E[2]};
        const double gn = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
        const double x1 = x0 + dt * un[0] / gn, y1 = y0 + dt * un[1] / gn, z1 = z0 + dt * un[2] / gn;
        const double r1 = sqrt(y1 * y1 + z1 * z1);
        if (!inside(x1 / h, r1 / dr)) {
            if (a.skipped) atomicAdd(a.skipped, 1ull);
            return false;
        }
        a.x[p] = x1; a.y[p] = y1; a.z[p] = z1;
        a.ux[p] = un[0]; a.uy[p] = un[1]; a.uz[p] = un[2];

        // ---- deposit along x^n -> x^{n+1}
        double wo[3], wn[3];
        const int ko = spline3(sx0, wo), kn = spline3(x1 / h, wn);
        ib = min(ko, kn) - 1;
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            gx[ko - 1 + u - ib] += wo[u];
            hx[kn - 1 + u - ib] += wn[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) hx[u] -= gx[u];
        double vo[3], vn[3];
        const int jo = spline3(sr0, vo), jn = spline3(r1 / dr, vn);
        jb = max(0, min(jo, jn) - 1);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            gr[fold_row(jo - 1 + v, false) - jb] += vo[v];
            hr[fold_row(jn - 1 + v, false) - jb] += vn[v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) hr[v] -= gr[v];
        dth = atan2(z1, y1) - th0;
        dth -= 2.0 * kPi * floor((dth + kPi) / (2.0 * kPi));
        const double Q = a.q ? a.q[p] : a.charge;
        qdt = Q / dt;
        kth = Q * dth / (2.0 * kPi * h * dr * dt);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = jb + v;
            ax_[v] = 2.0 * kPi * (j == 0 ? dr / 8.0 : j * dr) * dr;   // A_{r theta, j}
            ar_[v] = 2.0 * kPi * (j + 0.5) * dr * h;                  // A_{x theta, j+1/2}
        }
        return true;
    };
    const bool active = prep();

    // The workgroup's deposit windows (4 x 4 cells from (jb, ib)) span a box
    // of rows [j0, j1 + 4) and columns [i0, i1 + 4).  When it fits the tile
    // (particles sorted by cell: a few columns of consecutive rows), each mode
    // is accumulated there with LDS atomics and then added to the planes with
    // one global atomic per nonzero value; otherwise every value goes to the
    // planes directly.  The decision is uniform over the workgroup.
    __shared__ cx<T> tile[3 * kTileCells<T>];
    __shared__ int box[4];
    if (threadIdx.x == 0) {
        box[0] = 0x7fffffff; box[1] = -1; box[2] = 0x7fffffff; box[3] = -1;
    }
    __syncthreads();
    if (active) {
        atomicMin(&box[0], ib); atomicMax(&box[1], ib);
        atomicMin(&box[2], jb); atomicMax(&box[3], jb);
    }
    __syncthreads();
    const int i0 = box[0], j0 = box[2];
    const int tw = box[1] - i0 + 4, tht = box[3] - j0 + 4;   // tile width and height
    const bool tiled = box[1] >= 0 && tw * tht <= kTileCells<T>;
    const int tn = tiled ? tw * tht : 0;
    cx<T>* const planes[3] = {a.jx, a.jr, a.jt};
    auto add = [&](cx<T>* P, int m, int row, int col, cx<double> val) {
        if (val.re == 0.0 && val.im == 0.0) return;
        if (tiled) {
            const int k = P == a.jx ? 0 : (P == a.jr ? 1 : 2);
            cx<T>* e = tile + k * tn + (row - j0) * tw + (col - i0);
            atomicAdd(&e->re, T(val.re));
            atomicAdd(&e->im, T(val.im));
            return;
        }
        cx<T>* e = P + g.at(m, row, col);
        atomicAdd(&e->re, T(val.re));
        atomicAdd(&e->im, T(val.im));
    };
#pragma unroll 1
    for (int m = 0; m < M; ++m) {
        if (tiled) {
            for (int e = threadIdx.x; e < 3 * tn; e += blockDim.x) tile[e] = cx<T>{T(0), T(0)};
            __syncthreads();
        }
        if (active) {
            cx<double> Ek[3];
            moments(m * dth, Ek);
            double sc, cc;
            sincos(m * th0, &sc, &cc);
            const cx<double> C = m == 0 ? cx<double>{1.0, 0.0} : cx<double>{2.0 * cc, 2.0 * sc};
            for (int k = 0; k < 3; ++k) Ek[k] = C * Ek[k];
            // j_x: cumulative over the columns of each row (face x_{i+1/2})
#pragma unroll 1
            for (int v = 0; v < 4; ++v) {
                cx<double> acc{0.0, 0.0};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const cx<double> avg = gr[v] * Ek[0] + hr[v] * Ek[1];
                    acc = acc - (qdt * hx[u] / ax_[v]) * avg;
                    add(a.jx, m, jb + v, ib + u, acc);
                }
            }
            // j_r: cumulative outward over the rows of each column (face r_{j+1/2})
#pragma unroll 1
            for (int u = 0; u < 4; ++u) {
                cx<double> flux{0.0, 0.0};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const cx<double> avg = gx[u] * Ek[0] + hx[u] * Ek[1];
                    flux = flux - (qdt * hr[v]) * avg;
                    add(a.jr, m, jb + v, ib + u, (1.0 / ar_[v]) * flux);
                }
            }
            // j_theta at (x_i, r_j)
#pragma unroll 1
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const cx<double> avg = (gx[u] * gr[v]) * Ek[0] + (gx[u] * hr[v] + hx[u] * gr[v]) * Ek[1] +
                                           (hx[u] * hr[v]) * Ek[2];
                    add(a.jt, m, jb + v, ib + u, kth * avg);
                }
        }
        if (tiled) {
            __syncthreads();
            for (int e = threadIdx.x; e < 3 * tn; e += blockDim.x) {
                const cx<T> v = tile[e];
                if (v.re == T(0) && v.im == T(0)) continue;
                const int k = e / tn, c = e - k * tn;
                cx<T>* d = planes[k] + g.at(m, j0 + c / tw, i0 + c % tw);
                atomicAdd(&d->re, v.re);
                atomicAdd(&d->im, v.im);
            }
            __syncthreads();
        }
    }
}

template <typename T>
hipError_t particle_step(const PartArgs<T>& a, int M, hipStream_t s) {
    const dim3 blk(256);
    const dim3 grd(unsigned((a.count + 255) / 256));
    switch (M) {
#define QDS_PS(MM) case MM: hipLaunchKernelGGL((k_particle_step<T, MM>), grd, blk, 0, s, a); break;
        QDS_PS(1) QDS_PS(2) QDS_PS(3) QDS_PS(4) QDS_PS(5) QDS_PS(6) QDS_PS(7) QDS_PS(8)
#undef QDS_PS
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Zeroes three current planes of n 8-byte words each (a fill kernel rather
// than a memset node, so that the call may sit in a captured graph).
__global__ void k_zero_planes(uint2* a, uint2* b, uint2* c, size_t n) {
    const uint2 z = make_uint2(0u, 0u);
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
        a[i] = z;
        b[i] = z;
        c[i] = z;
    }
}

}  // namespace pic
}  // namespace qds

namespace {

template <typename T>
qds_status run(qds_ctx* h, const qds_state* st, int32_t extrapolate, qds_particles* pp, void* jx, void* jr, void* jt,
               unsigned long long* skipped, hipStream_t s) {
    qds::cx<T>* U[QDS_NPLANES];
    qds::cx<T>* V[QDS_NPLANES];
    plane_table<T>(h, st->buf[st->cur], U);
    plane_table<T>(h, st->buf[1 - st->cur], V);
    qds::pic::PartArgs<T> a{};
    a.g = geo(h);
    a.trp = U[QDS_P_TRP]; a.trm = U[QDS_P_TRM]; a.ttp = U[QDS_P_TTP]; a.ttm = U[QDS_P_TTM];
    a.ex = U[QDS_P_EX]; a.bx = U[QDS_P_BX];
    a.exq = extrapolate ? V[QDS_P_EX] : nullptr;
    a.bxq = extrapolate ? V[QDS_P_BX] : nullptr;
    a.x = pp->x; a.y = pp->y; a.z = pp->z;
    a.ux = pp->ux; a.uy = pp->uy; a.uz = pp->uz;
    a.q = pp->q;
    a.charge = pp->charge;
    a.qm = pp->qm;
    a.count = pp->count;
    a.jx = static_cast<qds::cx<T>*>(jx);
    a.jr = static_cast<qds::cx<T>*>(jr);
    a.jt = static_cast<qds::cx<T>*>(jt);
    a.skipped = skipped;
    if (pp->clear) {
        // every plane is plane_elems complex values of elem_bytes (8 or 16) bytes
        const size_t words = h->plane_elems * h->elem_bytes / 8;
        const unsigned blocks = unsigned(std::min<size_t>((words + 255) / 256, 4096));
        hipLaunchKernelGGL(qds::pic::k_zero_planes, dim3(blocks), dim3(256), 0, s, static_cast<uint2*>(jx),
                           static_cast<uint2*>(jr), static_cast<uint2*>(jt), words);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(h, QDS_EHIP, "clearing the current planes failed: %s", hipGetErrorString(e));
    }
    if (pp->count == 0) return QDS_OK;
    const hipError_t e = qds::pic::particle_step<T>(a, h->M, s);
    if (e != hipSuccess) return fail(h, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    return QDS_OK;
}

}  // namespace

extern "C" qds_status qds_particles_step(qds_handle h, const qds_state* fields, int32_t extrapolate,
                                         qds_particles* particles, void* jx, void* jr, void* jt,
                                         unsigned long long* skipped_dev, void* stream) {
    if (!h) return fail(nullptr, QDS_EINVAL, "null handle%s");
    qds_status s = check_state(h, fields);
    if (s != QDS_OK) return s;
    if (!particles || !jx || !jr || !jt) return fail(h, QDS_EINVAL, "null argument%s");
    if (particles->count < 0) return fail(h, QDS_EINVAL, "negative particle count%s");
    if (particles->count > 0 && (!particles->x || !particles->y || !particles->z || !particles->ux ||
                                 !particles->uy || !particles->uz))
        return fail(h, QDS_EINVAL, "null particle array%s");
    if (h->g.x_bc != QDS_X_OPEN) return fail(h, QDS_EUNSUPPORTED, "particles need open x boundaries%s");
    if (particles->count > (int64_t(1) << 40)) return fail(h, QDS_EINVAL, "too many particles%s");
    if (h->g.dtype == QDS_F64)
        return run<double>(h, fields, extrapolate, particles, jx, jr, jt, skipped_dev, hipStream_t(stream));
    return run<float>(h, fields, extrapolate, particles, jx, jr, jt, skipped_dev, hipStream_t(stream));
}
