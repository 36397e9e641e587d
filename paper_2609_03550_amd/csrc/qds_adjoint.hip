// Adjoint (transposed, reverse-time) step of the staged QDS step.
//
// Every forward stage y = f(x) of qds_stages.hip has a twin here that runs
// the same loops and branches and, for each term of f, adds the transposed
// contribution to the adjoint of its input: over the real inner product
// <u, v> = Re sum conj(u) v, a term y += c x gives xbar += conj(c) ybar, a term
// y += c conj(x) gives xbar += c conj(ybar), y = Re(x) gives xbar += Re(ybar).
// Adjoints of the new state (buffer B) also collect the contributions of the
// later stages that read it, so the stages run in reverse order.  Inputs the
// forward step reads from several threads receive atomic adds.
#include "qds_stage_ops.hpp"
#include "qds_current_rows.hpp"

namespace qds {
namespace adj {

// ---------------------------------------------------------------------------
// scatter-add helpers mirroring the forward accessors
// ---------------------------------------------------------------------------
__device__ __forceinline__ void aadd(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void aadd(float* p, float v) { atomicAdd(p, v); }

template <typename T>
__device__ __forceinline__ void cadd(cx<T>* p, cx<T> v) {
    T* q = reinterpret_cast<T*>(p);
    if (v.re != T(0)) aadd(q, v.re);
    if (v.im != T(0)) aadd(q + 1, v.im);
}

// adjoint of ldx(p, g, m, row, c)
template <typename T>
__device__ __forceinline__ void addx(cx<T>* p, const Geo& g, int m, int row, int c, cx<T> v) {
    if (c < 0 || c >= g.nx) {
        if (!g.per) return;
        c = (c + g.nx) % g.nx;
    }
    cadd(p + g.at(m, row, c), v);
}

template <typename T>
struct SetBar {
    cx<T>* trp; cx<T>* trm; cx<T>* ttp; cx<T>* ttm; cx<T>* ex; cx<T>* bx; cx<T>* jx; cx<T>* jr; cx<T>* jt;
};

// adjoints of bth / er / eth / brr (B_theta, E_r from T_r; E_theta, B_r from T_theta)
template <typename T>
__device__ __forceinline__ void add_bth(const SetBar<T>& s, const Geo& g, int m, int k, int c, cx<T> v) {
    if (k == g.nr) {
        addx(s.trp, g, m, k, c, v);
        return;
    }
    addx(s.trp, g, m, k, c, T(0.5) * v);
    addx(s.trm, g, m, k, c, -(T(0.5) * v));
}
template <typename T>
__device__ __forceinline__ void add_er(const SetBar<T>& s, const Geo& g, int m, int k, int c, cx<T> v) {
    addx(s.trp, g, m, k, c, T(0.5) * v);
    addx(s.trm, g, m, k, c, T(0.5) * v);
}
template <typename T>
__device__ __forceinline__ void add_eth(const SetBar<T>& s, const Geo& g, int m, int j, int c, cx<T> v) {
    addx(s.ttp, g, m, j, c, T(0.5) * v);
    addx(s.ttm, g, m, j, c, T(0.5) * v);
}
template <typename T>
__device__ __forceinline__ void add_brr(const SetBar<T>& s, const Geo& g, int m, int j, int c, cx<T> v) {
    addx(s.ttp, g, m, j, c, T(0.5) * v);
    addx(s.ttm, g, m, j, c, -(T(0.5) * v));
}
// conj(i s) v = -i s v
template <typename T>
__device__ __forceinline__ cx<T> imul_c(T s, cx<T> v) { return imul(-s, v); }

template <typename T>
struct StageBar {
    Geo g;
    SetPtr<T> A, B;             // forward old / new state of this set
    SetBar<T> Ab, Bb;           // their adjoints
    cx<T>* jx_addb;             // adjoint of the extra currents (or null)
    cx<T>* jr_addb;
    cx<T>* jt_addb;
    int plasma;
    double wp2;
};

// adjoint of jx_total (plasma part lives in B.jx, extra current, drive = const)
template <typename T>
__device__ __forceinline__ void jx_total_bar(const StageBar<T>& a, int m, int j, int i, cx<T> v) {
    const Geo& g = a.g;
    int c = i;
    if (g.per) c = (i + g.nx) % g.nx;
    else if (i < 0 || i >= g.nx - 1) return;
    if (a.plasma) cadd(a.Bb.jx + g.at(m, j, c), v);
    if (a.jx_addb) cadd(a.jx_addb + g.at(m, j, c), v);
}
template <typename T>
__device__ __forceinline__ void jr_total_bar(const StageBar<T>& a, int m, int k, int i, cx<T> v) {
    const Geo& g = a.g;
    if (a.plasma) {
        addx(a.Bb.jr, g, m, k, i, T(0.5) * v);
        addx(a.Bb.jr, g, m, k, i + 1, T(0.5) * v);
    }
    if (a.jr_addb) cadd(a.jr_addb + g.at(m, k, i), v);
}
template <typename T>
__device__ __forceinline__ void jt_total_bar(const StageBar<T>& a, int m, int j, int i, cx<T> v) {
    const Geo& g = a.g;
    if (a.plasma) {
        addx(a.Bb.jt, g, m, j, i, T(0.5) * v);
        addx(a.Bb.jt, g, m, j, i + 1, T(0.5) * v);
    }
    if (a.jt_addb) cadd(a.jt_addb + g.at(m, j, i), v);
}

template <typename T>
__device__ __forceinline__ cx<T> ldv(const cx<T>* p, const Geo& g, int m, int row, int c) {
    if (c < 0 || c >= g.nx) {
        if (!g.per) return zero<T>();
        c = (c + g.nx) % g.nx;
    }
    return ld(p + g.at(m, row, c));
}

// adjoint of bx_new_at (B_x^{n+1/2} at K = k) for the adjoint value bb
template <typename T>
__device__ void bx_new_bar(const StageBar<T>& a, int m, int k, int i, cx<T> bb) {
    const Geo& g = a.g;
    const T dr = T(g.dr), h = T(g.h);
    const T rk = (T(k) + T(0.5)) * dr;
    cadd(a.Ab.bx + g.at(m, k, i), bb);
    cx<T> fx = h * bb;
    cx<T> eavg = -(T(1) / rk) * fx;
    cx<T> de = -fx;
    cx<T> erav = imul_c(-T(m) / rk, fx);
    cx<T> lo = T(0.25) * eavg - (T(1) / (T(2) * dr)) * de;
    cx<T> hi = T(0.25) * eavg + (T(1) / (T(2) * dr)) * de;
    add_eth(a.Ab, g, m, k, i, lo);
    add_eth(a.Ab, g, m, k, i + 1, lo);
    add_eth(a.Ab, g, m, k + 1, i, hi);
    add_eth(a.Ab, g, m, k + 1, i + 1, hi);
    add_er(a.Ab, g, m, k, i, T(0.5) * erav);
    add_er(a.Ab, g, m, k, i + 1, T(0.5) * erav);
}

// ---- combining scatter: contributions to two planes over two rows and the
// columns i, i+1 are collected in registers, and the column i+1 share is
// handed to the next lane (which holds column i+1) by a DPP shift, so each
// point receives one atomic add per row from a wave.  flush2x2 is called by
// every lane of a wave (uniform control flow); lanes without work hold zeros.
__device__ __forceinline__ double prev_lane(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float prev_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
template <typename T>
__device__ __forceinline__ cx<T> prev_lane(cx<T> v) {
    return cx<T>{prev_lane(v.re), prev_lane(v.im)};
}

// two planes, rows r0 and r0 + 1, columns i and i + 1
template <typename T>
struct Acc2x2 {
    cx<T> p[2][2], q[2][2];
    __device__ __forceinline__ Acc2x2() {
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) p[r][c] = q[r][c] = zero<T>();
    }
};

template <typename T>
__device__ __forceinline__ void flush2x2(const Geo& g, int m, int i, int lane, int r0, int rmax, cx<T>* P, cx<T>* Q,
                                         const Acc2x2<T>& A) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int row = r0 + r;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            cx<T>* pl = w ? Q : P;
            const cx<T> v0 = w ? A.q[r][0] : A.p[r][0];
            const cx<T> v1 = w ? A.q[r][1] : A.p[r][1];
            const cx<T> got = prev_lane(v1);                 // column i of this lane from lane - 1
            const cx<T> own = lane > 0 ? v0 + got : v0;
            if (row < 0 || row > rmax) continue;
            if (i < g.nx) cadd(pl + g.at(m, row, i), own);
            if (lane == 63 || (g.per && i == g.nx - 1)) addx(pl, g, m, row, i + 1, v1);
        }
    }
}

// ---- adjoint of k_ghost_bth
template <typename T>
__global__ void __launch_bounds__(64) k_ghost_bth_bar(StageBar<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;                   // one mode per grid row
    if (i >= g.nx || !g.open_r) return;
    const int N = g.nr;
    const T h = T(g.h), dr = T(g.dr);
    const T rN = T(N) * dr;
    const T kap = (dr - h) / (dr + h), cR = T(2) * h * dr / (dr + h);
    {
        cx<T> ob = ld(a.Bb.trp + g.at(m, N, i));
        // out = I0 + kap (G0 - I1) + cR rt
        cx<T> rt = cR * ob;
        cx<T> I0 = ob - (T(1) / (T(2) * rN)) * (T(0.5) * rt);
        cx<T> G0 = kap * ob - (T(1) / (T(2) * rN)) * (T(0.5) * rt);
        cx<T> I1 = -(kap * ob);
        cx<T> dxer = -(T(0.5) * rt);
        cx<T> jxi = T(0.5) * rt;
        cx<T> br = imul_c(-T(m) / (T(2) * rN), rt);
        add_bth(a.Ab, g, m, N - 1, i, I0);
        cadd(a.Ab.trp + g.at(m, N, i), G0);
        cadd(a.Bb.trp + g.at(m, N - 1, i), T(0.5) * I1);
        cadd(a.Bb.trm + g.at(m, N - 1, i), -(T(0.5) * I1));
        add_er(a.Ab, g, m, N - 1, i + 1, (T(1) / (T(2) * h)) * dxer);
        add_er(a.Ab, g, m, N - 1, i - 1, -((T(1) / (T(2) * h)) * dxer));
        jx_total_bar(a, m, N, i, T(0.5) * jxi);
        jx_total_bar(a, m, N, i - 1, T(0.5) * jxi);
        add_brr(a.Ab, g, m, N, i, br);
    }
}

// ---- adjoint of k_transverse
//
// One thread per point (i, j), one wave per row j.  The shifted transport
// adjoints have a single writer per point here and take a plain
// read-add-write; so do the B_x and E_x adjoints, which each thread gathers for
// its own point (the shares of the rows j-1 and j+1 are recomputed from their
// transport adjoints); the plasma j_r / j_theta adjoints (columns i, i+1) leave
// through the combining scatter.
template <typename T>
__device__ __forceinline__ void rmw(cx<T>* p, cx<T> v) {
    st(p, ld(p) + v);
}
// one row of the combining scatter: v0 into column i, v1 into column i+1
template <typename T>
__device__ __forceinline__ void flush_row2(const Geo& g, int m, int i, int lane, int row, cx<T>* P, cx<T> v0,
                                           cx<T> v1) {
    const cx<T> got = prev_lane(v1);
    const cx<T> own = lane > 0 ? v0 + got : v0;
    if (i < g.nx) cadd(P + g.at(m, row, i), own);
    if (lane == 63 || (g.per && i == g.nx - 1)) addx(P, g, m, row, i + 1, v1);
}
template <typename T>
__global__ void __launch_bounds__(256) k_transverse_bar(StageBar<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int lane = threadIdx.x;           // blockDim.x is one wave: a wave shares j
    if (j > g.nr) return;                   // uniform over the wave
    const bool in = i < g.nx;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = in && (g.per || i < g.nx - 1);   // (implies column i+1 exists)
    const int ir = g.per ? (i + 1) % g.nx : i + 1;
    const bool hasr = in && ir < g.nx;      // column i+1 exists
    const cx<T> zc = zero<T>();
    // T_theta rows without transport: the wall row, and the axis row for m != 1
    auto zero_row = [&](int row, int m) { return (!g.open_r && row == g.nr) || (row == 0 && m != 1); };
    for (int m = 0; m < g.M; ++m) {
        cx<T> jr0 = zc, jr1 = zc;           // plasma j_r adjoint, columns i, i+1 of row j
        cx<T> jt0 = zc, jt1 = zc;           // plasma j_theta adjoint, columns i, i+1 of row j
        cx<T> exb = zc, bxb = zc;           // E_x and B_x adjoints at this point
        // ---- T_r on K = j
        if (in && j < g.nr) {
            const cx<T> pb = hasr ? ld(a.Bb.trp + g.at(m, j, ir)) : zc;
            const cx<T> mb = ld(a.Bb.trm + g.at(m, j, i));
            if (hasr) {
                rmw(a.Ab.trp + g.at(m, j, i), pb);
                rmw(a.Ab.trm + g.at(m, j, ir), mb);
            }
            if (live) {
                const T rk = (T(j) + T(0.5)) * dr;
                const cx<T> gr = h * (pb + mb), pr = h * (pb - mb);
                bxb = bxb + imul_c(-T(m) / rk, gr);
                if (a.plasma) jr0 = jr1 = T(-0.5) * gr;
                if (a.jr_addb) rmw(a.jr_addb + g.at(m, j, i), -gr);
                exb = exb - (T(1) / dr) * pr;
            }
        }
        // ---- the E_x share of T_r on K = j - 1
        if (live && j >= 1 && j - 1 < g.nr) {
            const cx<T> pb = ld(a.Bb.trp + g.at(m, j - 1, ir));
            const cx<T> mb = ld(a.Bb.trm + g.at(m, j - 1, i));
            exb = exb + (T(1) / dr) * (h * (pb - mb));
        }
        // ---- T_theta on J = j
        if (in && !zero_row(j, m)) {
            const cx<T> pb = ld(a.Bb.ttp + g.at(m, j, i));
            const cx<T> mb = hasr ? ld(a.Bb.ttm + g.at(m, j, ir)) : zc;
            if (hasr) {
                rmw(a.Ab.ttp + g.at(m, j, ir), pb);
                rmw(a.Ab.ttm + g.at(m, j, i), mb);
            }
            if (live) {
                const cx<T> gt = h * (pb + mb), pt = h * (pb - mb);
                if (j == 0) {
                    // (on the axis only mode 1 gets here: its axis relation; its
                    // E_x share goes to row 1, gathered there)
                    bxb = bxb - (T(2) / dr) * gt;
                } else {
                    const T rj = T(j) * dr;
                    bxb = bxb - (T(1) / dr) * gt;
                    exb = exb + imul_c(T(m) / rj, pt);
                }
                if (a.plasma) jt0 = jt1 = T(-0.5) * gt;
                if (a.jt_addb) rmw(a.jt_addb + g.at(m, j, i), -gt);
            }
        }
        // ---- the B_x share of T_theta on J = j + 1
        if (live && j + 1 <= g.nr && !zero_row(j + 1, m)) {
            const cx<T> pb = ld(a.Bb.ttp + g.at(m, j + 1, i));
            const cx<T> mb = ld(a.Bb.ttm + g.at(m, j + 1, ir));
            bxb = bxb + (T(1) / dr) * (h * (pb + mb));
        }
        // ---- the E_x share of the mode-1 axis relation on J = 0, at row 1
        if (live && j == 1 && m == 1) {
            const cx<T> pb = ld(a.Bb.ttp + g.at(m, 0, i));
            const cx<T> mb = ld(a.Bb.ttm + g.at(m, 0, ir));
            exb = exb + imul_c(T(1) / dr, h * (pb - mb));
        }
        if (exb.re != T(0) || exb.im != T(0)) rmw(a.Bb.ex + g.at(m, j, i), exb);
        if (bxb.re != T(0) || bxb.im != T(0)) rmw(a.Bb.bx + g.at(m, j, i), bxb);
        if (a.plasma) {
            if (j < g.nr) flush_row2(g, m, i, lane, j, a.Bb.jr, jr0, jr1);
            flush_row2(g, m, i, lane, j, a.Bb.jt, jt0, jt1);
        }
    }
}

// ---- adjoint of k_longitudinal
//
// One thread per point (i, j), one wave per row j over 63 columns (lane 0 is a
// halo: it computes column i-1 for lane 1 and writes nothing).  Every plane
// point has one writer: the point's own planes (E_x, B_x, the currents) take a
// plain read-add-write, and so do the transverse planes, whose values each
// thread gathers for its own point: the B_theta / E_r and B_r / E_theta
// stencils of E_x on J = j, j+1 and of B_x on K = j-1, j (the neighbouring
// rows' shares recomputed from their adjoints), the column i-1 shares from the
// previous lane by a DPP shift.  The exterior ghost row's B_x adjoint writes to
// points other threads own and runs afterwards in k_longitudinal_ghost_bar.
constexpr int kLongOwn = 63;
template <typename T>
__global__ void __launch_bounds__(256) k_longitudinal_bar(StageBar<T> a) {
    const Geo& g = a.g;
    const int lane = threadIdx.x;           // blockDim.x is one wave: a wave shares j
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (j > g.nr) return;                   // uniform over the wave
    const int raw = blockIdx.x * kLongOwn - 1 + lane;
    const int i = g.per ? ((raw % g.nx) + g.nx) % g.nx : min(max(raw, 0), g.nx - 1);
    const bool in = g.per || (raw >= 0 && raw < g.nx);    // a column of its own
    const bool owner = lane >= 1 && raw < g.nx;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = in && (g.per || i < g.nx - 1);
    const T wp2h = T(a.wp2 * g.h);
    const T half = T(0.5);
    const T i2dr = T(1) / (T(2) * dr);
    const bool wall_j = !g.open_r && j == g.nr;           // E_x and T_theta fixed on the wall row
    const bool wall_j1 = !g.open_r && j + 1 == g.nr;
    for (int m = 0; m < g.M; ++m) {
        const size_t e = g.at(m, j, i);
        // stencil values of this column's cell, which go to the columns i and i+1 alike
        cx<T> Sp = zero<T>(), Sq = zero<T>();     // T_r^+, T_r^- on K row j
        cx<T> Tp = zero<T>(), Tq = zero<T>();     // T_theta^+, T_theta^- on J row j
        cx<T> Op = zero<T>(), Oq = zero<T>();     // T_r^+- of this column only (plasma)
        cx<T> Up = zero<T>(), Uq = zero<T>();     // T_theta^+- of this column only (plasma)
        // B_theta / E_r into K row j (the exterior ghost row holds B_theta in T_r^+)
        auto bth = [&](cx<T> v) {
            if (j == g.nr) {
                Sp = Sp + v;
                return;
            }
            Sp = Sp + half * v;
            Sq = Sq - half * v;
        };
        if (in) {
            cx<T> exb = zero<T>();      // adjoint into A.ex at this point
            cx<T> jxh = zero<T>();      // adjoint of the total j_x at this point
            // ---- E_x on J = j: K row j (hi) and J row j (B_r)
            const cx<T> eb = ld(a.Bb.ex + e);
            if (live && !wall_j) {
                if (j == 0) {
                    if (m == 0) {
                        exb = exb + eb;
                        const cx<T> gx = h * eb;
                        bth(half * ((T(4) / dr) * gx));
                        jxh = jxh - gx;
                    }
                } else {
                    const T rj = T(j) * dr;
                    exb = exb + eb;
                    const cx<T> gx = h * eb;
                    jxh = jxh - gx;
                    bth(T(0.25) * ((T(1) / rj) * gx) + i2dr * gx);
                    const cx<T> brav = half * imul_c(T(m) / rj, gx);
                    Tp = Tp + half * brav;
                    Tq = Tq - half * brav;
                }
            }
            // ---- E_x on J = j+1: its K row j share (lo)
            if (live && j + 1 <= g.nr && !wall_j1) {
                const cx<T> gx = h * ld(a.Bb.ex + g.at(m, j + 1, i));
                const T rj = T(j + 1) * dr;
                const cx<T> lo = T(0.25) * ((T(1) / rj) * gx) - i2dr * gx;
                Sp = Sp + half * lo;
                Sq = Sq - half * lo;
            }
            if (owner && a.jx_addb && (jxh.re != T(0) || jxh.im != T(0))) rmw(a.jx_addb + e, jxh);
            // ---- B_x on K = j: J row j (lo) and K row j (E_r); its J row j+1 share is gathered there
            if (j < g.nr && live) {
                const cx<T> bb = ld(a.Bb.bx + e);
                const T rk = (T(j) + T(0.5)) * dr;
                if (owner) rmw(a.Ab.bx + e, bb);
                const cx<T> fx = h * bb;
                const cx<T> lo = T(0.25) * (-(T(1) / rk) * fx) + i2dr * fx;
                Tp = Tp + half * lo;
                Tq = Tq + half * lo;
                const cx<T> erav = half * imul_c(-T(m) / rk, fx);
                Sp = Sp + half * erav;
                Sq = Sq + half * erav;
            }
            // ---- B_x on K = j-1: its J row j share (hi)
            if (j >= 1 && j - 1 < g.nr && live) {
                const cx<T> fx = h * ld(a.Bb.bx + g.at(m, j - 1, i));
                const T rk = (T(j) - T(0.5)) * dr;
                const cx<T> hi = T(0.25) * (-(T(1) / rk) * fx) - i2dr * fx;
                Tp = Tp + half * hi;
                Tq = Tq + half * hi;
            }
            // ---- plasma response
            if (a.plasma) {
                const cx<T> jxb = ld(a.Bb.jx + e) + jxh;
                if (owner) rmw(a.Ab.jx + e, jxb);
                exb = exb + wp2h * jxb;
                if (j < g.nr) {
                    const cx<T> jrb = ld(a.Bb.jr + e);
                    if (owner) rmw(a.Ab.jr + e, jrb);
                    Op = Op + half * (wp2h * jrb);
                    Oq = Oq + half * (wp2h * jrb);
                }
                if (!wall_j) {
                    const cx<T> jtb = ld(a.Bb.jt + e);
                    if (owner) rmw(a.Ab.jt + e, jtb);
                    Up = Up + half * (wp2h * jtb);
                    Uq = Uq + half * (wp2h * jtb);
                }
            }
            if (owner && (exb.re != T(0) || exb.im != T(0))) rmw(a.Ab.ex + e, exb);
        }
        // column i: this cell's stencil, the previous column's, and this column's own terms
        const cx<T> rp = Sp + prev_lane(Sp) + Op, rq = Sq + prev_lane(Sq) + Oq;
        const cx<T> tp = Tp + prev_lane(Tp) + Up, tq = Tq + prev_lane(Tq) + Uq;
        if (owner) {
            if (rp.re != T(0) || rp.im != T(0)) rmw(a.Ab.trp + e, rp);
            if (rq.re != T(0) || rq.im != T(0)) rmw(a.Ab.trm + e, rq);
            if (tp.re != T(0) || tp.im != T(0)) rmw(a.Ab.ttp + e, tp);
            if (tq.re != T(0) || tq.im != T(0)) rmw(a.Ab.ttm + e, tq);
        }
    }
}

// ---- adjoint of the exterior ghost B_x of k_longitudinal (row nr), after k_longitudinal_bar
template <typename T>
__global__ void __launch_bounds__(64) k_longitudinal_ghost_bar(StageBar<T> a) {
    const Geo& g = a.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;                   // one mode per grid row
    if (i >= g.nx || !g.open_r) return;
    if (!(g.per || i < g.nx - 1)) return;
    const int N = g.nr;
    const T h = T(g.h), dr = T(g.dr);
    const T rN = T(N) * dr;
    const T kap = (dr - h) / (dr + h), cR = T(2) * h * dr / (dr + h);
    const T wp2h = T(a.wp2 * g.h);
    {
        cx<T> gh = ld(a.Bb.bx + g.at(m, N, i));
        cadd(a.Ab.bx + g.at(m, N - 1, i), gh);
        cadd(a.Ab.bx + g.at(m, N, i), kap * gh);
        bx_new_bar(a, m, N - 1, i, -(kap * gh));
        cx<T> rx = cR * gh;
        add_brr(a.Ab, g, m, N, i + 1, (T(0.5) / h) * rx);
        add_brr(a.Ab, g, m, N, i, -((T(0.5) / h) * rx));
        cx<T> ea = -(T(1) / (T(2) * rN)) * rx;
        add_eth(a.Ab, g, m, N, i, T(0.5) * ea);
        add_eth(a.Ab, g, m, N, i + 1, T(0.5) * ea);
        cx<T> ra = imul_c(-T(m) / (T(2) * rN), rx);
        add_er(a.Ab, g, m, N - 1, i, T(0.5) * ra);
        add_er(a.Ab, g, m, N - 1, i + 1, T(0.5) * ra);
        cx<T> jt = -(T(0.5) * rx);
        if (a.plasma) {
            addx(a.Ab.jt, g, m, N, i, T(0.5) * jt);
            add_eth(a.Ab, g, m, N, i, wp2h * (T(0.5) * jt));
            if (g.per || i + 1 < g.nx) {
                addx(a.Ab.jt, g, m, N, i + 1, T(0.5) * jt);
                add_eth(a.Ab, g, m, N, i + 1, wp2h * (T(0.5) * jt));
            }
        }
        if (a.jt_addb) cadd(a.jt_addb + g.at(m, N, i), jt);
    }
}

// ---------------------------------------------------------------------------
// mode convolution transpose: given the output adjoints Ob[m], add the
// adjoints of A and B (see conv_acc for the forward sums)
// ---------------------------------------------------------------------------
template <typename T, int M>
__device__ __forceinline__ void conv_bar(const cx<T>* A, const cx<T>* B, const cx<T>* Ob, T sign, cx<T>* Ab,
                                         cx<T>* Bb) {
    {
        cx<T> o = sign * Ob[0];
        // A0 B0
        Ab[0] = Ab[0] + conj(B[0]) * o;
        Bb[0] = Bb[0] + conj(A[0]) * o;
        // 1/2 Re(A_k conj(B_k)) added to the real part
#pragma unroll
        for (int k = 1; k < M; ++k) {
            Ab[k] = Ab[k] + (T(0.5) * o.re) * B[k];
            Bb[k] = Bb[k] + (T(0.5) * o.re) * A[k];
        }
    }
#pragma unroll
    for (int m = 1; m < M; ++m) {
        cx<T> o = (sign * T(0.5)) * Ob[m];
#pragma unroll
        for (int k = 0; k < M; ++k) {
#pragma unroll
            for (int l = 0; l < M; ++l) {
                if (k + l == m) {           // A_k B_l
                    Ab[k] = Ab[k] + conj(B[l]) * o;
                    Bb[l] = Bb[l] + conj(A[k]) * o;
                }
                if (k - l == m) {           // A_k conj(B_l)
                    Ab[k] = Ab[k] + B[l] * o;
                    Bb[l] = Bb[l] + A[k] * conj(o);
                }
                if (l - k == m) {           // conj(A_k) B_l
                    Ab[k] = Ab[k] + B[l] * conj(o);
                    Bb[l] = Bb[l] + A[k] * o;
                }
            }
        }
    }
}

template <typename T>
struct AxBar {
    AxionArgs<T> f;             // forward values
    SetBar<T> A0b, B0b;         // adjoints of the background set, old / new
    cx<T>* phiAb; cx<T>* tapAb; cx<T>* tamAb;
    cx<T>* phiBb; cx<T>* tapBb; cx<T>* tamBb;
    cx<T>* jaxb; cx<T>* jarb; cx<T>* jatb;
    double* dLds;               // [2]: dL/ds_phi, dL/ds_j accumulated
};

// ---- adjoint of k_axion_phi
template <typename T>
__global__ void __launch_bounds__(256) k_axion_phi_bar(AxBar<T> a) {
    // one thread per half point (i, k), one wave per row k: the phi adjoints of
    // the point (and of the exterior ghost row, from k = nr - 1 only) have one
    // writer (plain read-add-write); the T_a^+- shares of the columns i, i+1
    // are combined across lanes before one atomic add per point
    const Geo& g = a.f.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y * blockDim.y + threadIdx.y;
    const int lane = threadIdx.x;               // blockDim.x is one wave: a wave shares k
    if (k >= g.nr) return;                      // uniform over the wave
    const bool in = i < g.nx;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = in && (g.per || i < g.nx - 1);
    const T kap = (dr - h) / (dr + h);
    for (int m = 0; m < g.M; ++m) {
        cx<T> q = zero<T>();
        if (in) {
            cx<T> pb = ld(a.phiBb + g.at(m, k, i));
            cx<T> own = zero<T>();
            if (k == g.nr - 1) {
                const cx<T> Gb = ld(a.phiBb + g.at(m, g.nr, i));
                if (g.open_r) {
                    if (live) {
                        own = own + Gb;
                        rmw(a.phiAb + g.at(m, g.nr, i), kap * Gb);
                        pb = pb - kap * Gb;
                    }
                } else {
                    rmw(a.phiAb + g.at(m, g.nr, i), Gb);
                }
            }
            if (live) {
                own = own + pb;
                q = (h / T(4)) * pb;
            }
            if (own.re != T(0) || own.im != T(0)) rmw(a.phiAb + g.at(m, k, i), own);
        }
        flush_row2(g, m, i, lane, k, a.tapBb, q, q);
        flush_row2(g, m, i, lane, k, a.tamBb, q, q);
    }
}

// block reduction of one double per thread into acc (one atomic per block)
__device__ __forceinline__ void block_sum_add(double v, double* acc) {
    __shared__ double red[256];
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
    const int n = blockDim.x * blockDim.y;
    red[t] = v;
    __syncthreads();
    for (int s = n / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0 && red[0] != 0.0) atomicAdd(acc, red[0]);
}

// ---- adjoint of k_axion_ta (S_a, Gamma_a, T_a shift)
//
// One thread per half point (i, k), one wave per row k.  The T_a shift
// adjoints and the point's own B_x adjoints have a single writer here (plain
// read-add-write); the transverse stencils of the source leave through the
// combining scatter; phi and E_x (rows k-1..k+1) take atomic adds.
template <typename T, int M>
__global__ void __launch_bounds__(256) k_axion_ta_bar(AxBar<T> a) {
    const Geo& g = a.f.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y * blockDim.y + threadIdx.y;
    const int lane = threadIdx.x;           // blockDim.x is one wave: a wave shares k
    const bool inb = i < g.nx && k < g.nr;
    const T h = T(g.h), dr = T(g.dr);
    const bool live = inb && (g.per || i < g.nx - 1);
    const int ir = g.per ? (i + 1) % g.nx : i + 1;
    const bool hasr = inb && ir < g.nx;
    const AxionArgs<T>& f = a.f;
    const T half = T(0.5);
    double dsphi = 0.0;
    cx<T> gab[M];
#pragma unroll
    for (int m = 0; m < M; ++m) gab[m] = zero<T>();
    if (inb) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const cx<T> tp = hasr ? ld(a.tapBb + g.at(m, k, ir)) : zero<T>();
            const cx<T> tm = ld(a.tamBb + g.at(m, k, i));
            if (hasr) {
                rmw(a.tapAb + g.at(m, k, i), tp);
                rmw(a.tamAb + g.at(m, k, ir), tm);
            }
            gab[m] = h * (tp + tm);
        }
    }
    cx<T> Exb[M], Bxb[M], Erb[M], Brb[M], Etb[M], Btb[M];
#pragma unroll
    for (int m = 0; m < M; ++m) Exb[m] = Bxb[m] = Erb[m] = Brb[m] = Etb[m] = Btb[m] = zero<T>();
    if (live) {
        const T rk = (T(k) + T(0.5)) * dr;
        cx<T> Sb[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            cx<T> gb = gab[m];
            // Gamma_a = Lap(phi) - (m^2/r^2 + m_a^2) phi + s_phi S
            cadd(a.phiAb + g.at(m, k, i), (-T(2) / (dr * dr) - (T(m * m) / (rk * rk) + T(f.ma2))) * gb);
            cx<T> cu = (T(1) / (dr * dr) + T(1) / (T(2) * dr * rk)) * gb;
            if (k + 1 < g.nr) cadd(a.phiAb + g.at(m, k + 1, i), cu);
            else if (g.open_r) cadd(a.phiAb + g.at(m, g.nr, i), cu);
            if (k > 0) cadd(a.phiAb + g.at(m, k - 1, i), (T(1) / (dr * dr) - T(1) / (T(2) * dr * rk)) * gb);
            Sb[m] = T(f.s_phi) * gb;
        }
        // recompute the forward source factors
        cx<T> Ex[M], Bx[M], Er[M], Br[M], Et[M], Bt[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            Er[m] = T(0.5) * (er(f.A0, g, m, k, i) + er(f.A0, g, m, k, i + 1));
            Bt[m] = T(0.5) * (bth(f.A0, g, m, k, i) + bth(f.A0, g, m, k, i + 1));
            Et[m] = T(0.25) * (eth(f.A0, g, m, k, i) + eth(f.A0, g, m, k + 1, i) + eth(f.A0, g, m, k, i + 1) +
                               eth(f.A0, g, m, k + 1, i + 1));
            Br[m] = T(0.25) * (brr(f.A0, g, m, k, i) + brr(f.A0, g, m, k + 1, i) + brr(f.A0, g, m, k, i + 1) +
                               brr(f.A0, g, m, k + 1, i + 1));
            cx<T> e0 = T(0.5) * (ld(f.A0.ex + g.at(m, k, i)) + ld(f.B0.ex + g.at(m, k, i)));
            cx<T> e1 = T(0.5) * (ld(f.A0.ex + g.at(m, k + 1, i)) + ld(f.B0.ex + g.at(m, k + 1, i)));
            Ex[m] = T(0.5) * (e0 + e1);
            Bx[m] = T(0.5) * (ld(f.A0.bx + g.at(m, k, i)) + ld(f.B0.bx + g.at(m, k, i)));
        }
        Bx[0] = Bx[0] + f.bx0;
        if (M > 1) {
            Br[1] = Br[1] + f.br1;
            Bt[1] = Bt[1] + f.bt1;
        }
        if (a.dLds) {
            cx<T> S[M];
#pragma unroll
            for (int m = 0; m < M; ++m) S[m] = zero<T>();
            conv_acc<T, M>(Ex, Bx, T(1), S);
            conv_acc<T, M>(Er, Br, T(1), S);
            conv_acc<T, M>(Et, Bt, T(1), S);
#pragma unroll
            for (int m = 0; m < M; ++m) dsphi += double(gab[m].re * S[m].re + gab[m].im * S[m].im);
        }
        conv_bar<T, M>(Ex, Bx, Sb, T(1), Exb, Bxb);
        conv_bar<T, M>(Er, Br, Sb, T(1), Erb, Brb);
        conv_bar<T, M>(Et, Bt, Sb, T(1), Etb, Btb);
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        Acc2x2<T> R;    // T_r^+ (p), T_r^- (q) on the half row k (slot 0)
        Acc2x2<T> Q;    // T_theta^+ (p), T_theta^- (q) on the rows k (slot 0), k+1 (slot 1)
        if (live) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // E_r and B_theta averaged over the columns i, i+1
                const cx<T> e = half * (half * Erb[m]), b = half * (half * Btb[m]);
                R.p[0][c] = R.p[0][c] + e + b;
                R.q[0][c] = R.q[0][c] + e - b;
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    // E_theta and B_r averaged over the rows k, k+1 and the columns
                    const cx<T> et = half * (T(0.25) * Etb[m]), br = half * (T(0.25) * Brb[m]);
                    Q.p[r][c] = Q.p[r][c] + et + br;
                    Q.q[r][c] = Q.q[r][c] + et - br;
                }
            }
            const cx<T> ex = T(0.25) * Exb[m];
            cadd(a.A0b.ex + g.at(m, k, i), ex);
            cadd(a.B0b.ex + g.at(m, k, i), ex);
            cadd(a.A0b.ex + g.at(m, k + 1, i), ex);
            cadd(a.B0b.ex + g.at(m, k + 1, i), ex);
            const cx<T> bx = T(0.5) * Bxb[m];
            rmw(a.A0b.bx + g.at(m, k, i), bx);
            rmw(a.B0b.bx + g.at(m, k, i), bx);
        }
        if (k < g.nr) {
            flush2x2(g, m, i, lane, k, g.nr - 1, a.A0b.trp, a.A0b.trm, R);
            flush2x2(g, m, i, lane, k, g.nr, a.A0b.ttp, a.A0b.ttm, Q);
        }
    }
    if (a.dLds) block_sum_add(dsphi, a.dLds);
}

// ---- adjoint of ja_factors for one cell: the 18 factor adjoints of mode m
// into the adjoints of the planes they read, with the combining scatter
template <typename T>
__device__ void ja_factors_bar_comb(const AxBar<T>& a, int m, int i, int j, int lane, const cx<T>* fb) {
    const AxionArgs<T>& f = a.f;
    const Geo& g = f.g;
    const T dr = T(g.dr);
    const bool ax = (j == 0);
    const T rj = T(j) * dr;
    const T rk = (T(j) + T(0.5)) * dr;
    const T r_half = T(0.5) * dr;
    const T par = parity<T>(m);
    const T tg = tghost<T>(m);
    const T h = T(0.5);
    // ---- T_r at the old and new levels (half rows j-1, j): E_r -> (+1/2, +1/2), B_theta -> (+1/2, -1/2)
    {
        Acc2x2<T> A, B;
        const cx<T> q2 = T(0.25) * fb[2];
        const cx<T> q = T(0.25) * fb[6], qe = T(0.25) * fb[10];
        for (int cc = 0; cc < 2; ++cc) {
            // f2: E_r^n of j_a,x
            cx<T> eb = q2, gb = q2;
            if (ax) eb = eb + tg * gb;
            else { A.p[0][cc] = A.p[0][cc] + h * gb; A.q[0][cc] = A.q[0][cc] + h * gb; }
            A.p[1][cc] = A.p[1][cc] + h * eb; A.q[1][cc] = A.q[1][cc] + h * eb;
            // f6 (B_theta) and f10 (E_r) of j_a,theta, both levels
            cx<T> bb = q, gbb = q, ebb = qe, gebb = qe;
            if (ax) {
                bb = bb + tg * gbb;
                ebb = ebb + tg * gebb;
            } else {
                const cx<T> tp = h * (h * gbb) + h * (h * gebb), tm = h * (h * gebb) - h * (h * gbb);
                A.p[0][cc] = A.p[0][cc] + tp; A.q[0][cc] = A.q[0][cc] + tm;
                B.p[0][cc] = B.p[0][cc] + tp; B.q[0][cc] = B.q[0][cc] + tm;
            }
            const cx<T> tp = h * (h * bb) + h * (h * ebb), tm = h * (h * ebb) - h * (h * bb);
            A.p[1][cc] = A.p[1][cc] + tp; A.q[1][cc] = A.q[1][cc] + tm;
            B.p[1][cc] = B.p[1][cc] + tp; B.q[1][cc] = B.q[1][cc] + tm;
        }
        flush2x2(g, m, i, lane, j - 1, g.nr - 1, a.A0b.trp, a.A0b.trm, A);
        flush2x2(g, m, i, lane, j - 1, g.nr - 1, a.B0b.trp, a.B0b.trm, B);
    }
    // ---- T_theta at both levels (rows j, j+1; the m = 1 axis terms on row 0):
    // E_theta -> (+1/2, +1/2), B_r -> (+1/2, -1/2)
    {
        Acc2x2<T> A, B;
        auto eth = [&](Acc2x2<T>& X, int r, int cc, cx<T> v) {
            X.p[r][cc] = X.p[r][cc] + h * v; X.q[r][cc] = X.q[r][cc] + h * v;
        };
        auto brr = [&](Acc2x2<T>& X, int r, int cc, cx<T> v) {
            X.p[r][cc] = X.p[r][cc] + h * v; X.q[r][cc] = X.q[r][cc] - h * v;
        };
        // f4: E_theta^n(j) averaged over the columns
        eth(A, 0, 0, h * fb[4]);
        eth(A, 0, 1, h * fb[4]);
        if (ax && m == 1) {
            const cx<T> q2 = T(0.25) * fb[2], q = T(0.25) * fb[6], qe = T(0.25) * fb[10];
            for (int cc = 0; cc < 2; ++cc) {
                eth(A, 0, cc, imul_c(T(2), q2));                 // f2 axis: g = 2i E_th(0) - e
                const cx<T> brb = imul_c(-T(2), q);               // f6 axis: gb = -2i br - b
                brr(A, 0, cc, h * brb);
                brr(B, 0, cc, h * brb);
                const cx<T> etb = imul_c(T(2), qe);               // f10 axis: ge = 2i et - e
                eth(A, 0, cc, h * etb);
                eth(B, 0, cc, h * etb);
            }
        }
        // f12 (B_r) and f14 (E_theta) of j_a,r over rows j, j+1 and both columns
        const cx<T> sb = T(0.25) * fb[12], se = T(0.25) * fb[14];
        for (int dj = 0; dj < 2; ++dj)
            for (int cc = 0; cc < 2; ++cc) {
                brr(A, dj, cc, h * sb);
                brr(B, dj, cc, h * sb);
                eth(A, dj, cc, h * se);
                eth(B, dj, cc, h * se);
            }
        flush2x2(g, m, i, lane, j, g.nr, a.A0b.ttp, a.A0b.ttm, A);
        flush2x2(g, m, i, lane, j, g.nr, a.B0b.ttp, a.B0b.ttm, B);
    }
    // ---- T_a at t^{n-1/2} (A) and t^{n+1/2} (B), half rows j-1, j:
    // dto -> A (+1/2, +1/2), dth -> B (+1/2, +1/2), dxh -> B (-1/2, +1/2)
    {
        Acc2x2<T> A, B;
        auto dto = [&](int r, int cc, cx<T> v) { A.p[r][cc] = A.p[r][cc] + h * v; A.q[r][cc] = A.q[r][cc] + h * v; };
        auto dth = [&](int r, int cc, cx<T> v) { B.p[r][cc] = B.p[r][cc] + h * v; B.q[r][cc] = B.q[r][cc] + h * v; };
        auto dxh = [&](int r, int cc, cx<T> v) { B.p[r][cc] = B.p[r][cc] - h * v; B.q[r][cc] = B.q[r][cc] + h * v; };
        const cx<T> q = T(0.25) * fb[1];
        const cx<T> qt = T(0.25) * fb[7], qx = T(0.25) * fb[11];
        for (int cc = 0; cc < 2; ++cc) {
            // f1: d_t phi at t^n = (dto + dth)/2 on rows j-1, j
            cx<T> db = q, lb = q;
            if (ax) db = db + par * lb;
            dto(1, cc, h * db);
            dth(1, cc, h * db);
            if (!ax) { dto(0, cc, h * lb); dth(0, cc, h * lb); }
            // f7 (d_t phi) and f11 (d_x phi) at t^{n+1/2}
            cx<T> tb = qt, tlb = qt, xb = qx, xlb = qx;
            if (ax) { tb = tb + par * tlb; xb = xb + par * xlb; }
            else { dth(0, cc, tlb); dxh(0, cc, xlb); }
            dth(1, cc, tb);
            dxh(1, cc, xb);
            // f13, f15 of j_a,r (row j)
            dth(1, cc, h * fb[13]);
            dxh(1, cc, h * fb[15]);
        }
        flush2x2(g, m, i, lane, j - 1, g.nr - 1, a.tapAb, a.tamAb, A);
        flush2x2(g, m, i, lane, j - 1, g.nr - 1, a.tapBb, a.tamBb, B);
    }
    if (j >= g.nr || i >= g.nx) return;
    // ---- column-i planes: B_x (both levels), phi (both levels), E_x^{n+1/2}
    {
        // f0
        cx<T> hib = h * fb[0], lob = h * fb[0];
        if (ax) hib = hib + par * lob;
        cx<T> bx_hi = h * hib, bx_lo = ax ? zero<T>() : h * lob;
        // phi: f3, f5 (phiA), f9, f17 (both)
        cx<T> pA_hi = zero<T>(), pA_lo = zero<T>(), pB_hi = zero<T>(), pB_lo = zero<T>();
        if (ax) {
            if (m == 1) pA_hi = pA_hi + imul_c(-T(1) / r_half, fb[3]);
        } else {
            const cx<T> s3 = h * imul_c(-T(m) / rj, fb[3]);
            pA_hi = pA_hi + s3;
            pA_lo = pA_lo + s3;
        }
        {
            const cx<T> s5 = (T(1) / dr) * fb[5];
            cx<T> hi5 = s5, lo5 = -s5;
            if (ax) hi5 = hi5 + par * lo5;
            pA_hi = pA_hi + hi5;
            if (!ax) pA_lo = pA_lo + lo5;
        }
        {
            const cx<T> s9 = (T(1) / dr) * fb[9];
            cx<T> phb = s9, plb = -s9;
            if (ax) phb = phb + par * plb;
            pA_hi = pA_hi + h * phb; pB_hi = pB_hi + h * phb;
            if (!ax) { pA_lo = pA_lo + h * plb; pB_lo = pB_lo + h * plb; }
        }
        {
            const cx<T> ph = imul_c(-T(m) / rk, fb[17]);
            pA_hi = pA_hi + h * ph; pB_hi = pB_hi + h * ph;
        }
        cadd(a.A0b.bx + g.at(m, j, i), bx_hi);
        cadd(a.B0b.bx + g.at(m, j, i), bx_hi);
        cadd(a.phiAb + g.at(m, j, i), pA_hi);
        cadd(a.phiBb + g.at(m, j, i), pB_hi);
        if (!ax) {
            cadd(a.A0b.bx + g.at(m, j - 1, i), bx_lo);
            cadd(a.B0b.bx + g.at(m, j - 1, i), bx_lo);
            cadd(a.phiAb + g.at(m, j - 1, i), pA_lo);
            cadd(a.phiBb + g.at(m, j - 1, i), pB_lo);
        }
        // f8, f16
        cadd(a.B0b.ex + g.at(m, j, i), fb[8] + h * fb[16]);
        cadd(a.B0b.ex + g.at(m, j + 1, i), h * fb[16]);
    }
}

// ---- adjoint of k_axion_current
template <typename T, int M>
__global__ void __launch_bounds__(256) k_axion_current_bar(AxBar<T> a) {
    const Geo& g = a.f.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const bool inb = i < g.nx && j < g.nr;
    double dsj = 0.0;
    cx<T> Fb[18][M];
#pragma unroll
    for (int q = 0; q < 18; ++q)
#pragma unroll
        for (int m = 0; m < M; ++m) Fb[q][m] = zero<T>();
    if (inb && (g.per || i < g.nx - 1)) {
        const T sj = T(a.f.s_j);
        cx<T> F[18][M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            cx<T> f[18];
            ja_factors(a.f, m, i, j, f);
#pragma unroll
            for (int q = 0; q < 18; ++q) F[q][m] = f[q];
        }
        cx<T> jxb[M], jtb[M], jrb[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            jxb[m] = ld(a.jaxb + g.at(m, j, i));
            jtb[m] = ld(a.jatb + g.at(m, j, i));
            jrb[m] = ld(a.jarb + g.at(m, j, i));
        }
        if (a.dLds) {
            cx<T> jx[M], jt[M], jr[M];
#pragma unroll
            for (int m = 0; m < M; ++m) jx[m] = jt[m] = jr[m] = zero<T>();
            conv_acc<T, M>(F[0], F[1], T(1), jx);
            conv_acc<T, M>(F[2], F[3], T(-1), jx);
            conv_acc<T, M>(F[4], F[5], T(1), jx);
            conv_acc<T, M>(F[6], F[7], T(1), jt);
            conv_acc<T, M>(F[8], F[9], T(-1), jt);
            conv_acc<T, M>(F[10], F[11], T(1), jt);
            conv_acc<T, M>(F[12], F[13], T(1), jr);
            conv_acc<T, M>(F[14], F[15], T(-1), jr);
            conv_acc<T, M>(F[16], F[17], T(1), jr);
#pragma unroll
            for (int m = 0; m < M; ++m)
                dsj += double(jxb[m].re * jx[m].re + jxb[m].im * jx[m].im + jtb[m].re * jt[m].re +
                              jtb[m].im * jt[m].im + jrb[m].re * jr[m].re + jrb[m].im * jr[m].im);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            jxb[m] = sj * jxb[m];
            jtb[m] = sj * jtb[m];
            jrb[m] = sj * jrb[m];
        }
        conv_bar<T, M>(F[0], F[1], jxb, T(1), Fb[0], Fb[1]);
        conv_bar<T, M>(F[2], F[3], jxb, T(-1), Fb[2], Fb[3]);
        conv_bar<T, M>(F[4], F[5], jxb, T(1), Fb[4], Fb[5]);
        conv_bar<T, M>(F[6], F[7], jtb, T(1), Fb[6], Fb[7]);
        conv_bar<T, M>(F[8], F[9], jtb, T(-1), Fb[8], Fb[9]);
        conv_bar<T, M>(F[10], F[11], jtb, T(1), Fb[10], Fb[11]);
        conv_bar<T, M>(F[12], F[13], jrb, T(1), Fb[12], Fb[13]);
        conv_bar<T, M>(F[14], F[15], jrb, T(-1), Fb[14], Fb[15]);
        conv_bar<T, M>(F[16], F[17], jrb, T(1), Fb[16], Fb[17]);
    }
    // scatter in uniform control flow (the combining shifts need every lane);
    // rows at or beyond nr compute nothing
    if (j < g.nr) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            cx<T> fb[18];
#pragma unroll
            for (int q = 0; q < 18; ++q) fb[q] = Fb[q][m];
            ja_factors_bar_comb(a, m, i, j, int(threadIdx.x), fb);
        }
    }
    if (a.dLds) block_sum_add(dsj, a.dLds + 1);
}


// ---- adjoint of the marched axion current (qds_current.hip)
//
// Work layout of the forward march: a workgroup is M waves (one per mode) over
// a strip of 64 cells and a chunk of cell rows; lanes 1..62 own their column.
// For each cell row j a wave recomputes its mode's factors from the row window
// (qds_current_rows.hpp), exchanges the factors and its j_a adjoints with the
// other modes through LDS, forms the adjoints of its own mode's factors (the
// transpose of C_m) and transposes the factor expressions into adjoints of the
// window quantities.  Those of column i+1 go to the next lane by a DPP shift.
// After row j the K row j-1 and the J row j have all their contributions and
// are transposed into the planes: the old-level planes, which hold zero before
// this kernel, take a plain store in the rows inside the chunk and atomic adds
// in the rows the chunk shares with its neighbours; the new-level planes take
// one atomic add per point.
namespace curb {

using cur::FacC;
using cur::JRow;
using cur::KRow;
using cur::NbR;
using cur::NbT;
using cur::NbX;
constexpr int WAVE = cur::WAVE;
constexpr int OWN = 62;

template <typename T>
__device__ __forceinline__ void prev_add(cx<T>& acc, cx<T> v) {
    acc = acc + prev_lane(v);
}

// Ab, Bb of the own mode k of the adjoint of out_m += sign C_m{A, B} (all m),
// given Ob (the adjoint of out): the k-th entries of conv_bar
template <typename T, int M>
__device__ __forceinline__ void conv_bar_one(const cx<T>* A, const cx<T>* B, const cx<T>* Ob, T sign, int k,
                                             cx<T>& Ab, cx<T>& Bb) {
    {
        const cx<T> o = sign * Ob[0];
        if (k == 0) {
            Ab = Ab + cmul(B[0], o);
            Bb = Bb + cmul(A[0], o);
        } else {
#pragma unroll
            for (int q = 1; q < M; ++q)
                if (q == k) {
                    Ab = Ab + (T(0.5) * o.re) * B[q];
                    Bb = Bb + (T(0.5) * o.re) * A[q];
                }
        }
    }
#pragma unroll
    for (int m = 1; m < M; ++m) {
        const cx<T> o = (sign * T(0.5)) * Ob[m];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            // Ab[k]: terms A_k B_l (k + l = m), A_k conj(B_l) (k - l = m), conj(A_k) B_l (l - k = m)
            if (k + l == m) Ab = Ab + cmul(B[l], o);
            if (k - l == m) Ab = Ab + B[l] * o;
            if (l - k == m) Ab = Ab + mulc(B[l], o);
            // Bb[k]: terms A_l B_k (l + k = m), A_l conj(B_k) (l - k = m), conj(A_l) B_k (k - l = m)
            if (l + k == m) Bb = Bb + cmul(A[l], o);
            if (l - k == m) Bb = Bb + mulc(A[l], o);
            if (k - l == m) Bb = Bb + A[l] * o;
        }
    }
}

// transposes of cur::fac_x, fac_r, fac_t: factor adjoints b[6] into the
// adjoints of the window (kpb: K row j-1, kcb: K row j, jcb: J row j, jnb: J
// row j+1, n: the column-i+1 values)
template <typename T>
__device__ __forceinline__ void fac_x_bar(const FacC<T>& c, int j, const cx<T>* b, KRow<T>& kpb, KRow<T>& kcb,
                                          JRow<T>& jcb, NbX<T>& n) {
    const bool ax = j == 0;
    const int m = c.m;
    const T par = c.par;
    {
        const cx<T> q = T(0.5) * b[0];
        kcb.bxn = kcb.bxn + q;
        if (ax) kcb.bxn = kcb.bxn + par * q;
        else kpb.bxn = kpb.bxn + q;
    }
    {
        const cx<T> q = T(0.25) * b[1];
        kcb.dt0 = kcb.dt0 + q;
        n.dt1 = n.dt1 + q;
        if (ax) {
            kcb.dt0 = kcb.dt0 + par * q;
            n.dt1 = n.dt1 + par * q;
        } else {
            kpb.dt0 = kpb.dt0 + q;
            n.dtl1 = n.dtl1 + q;
        }
    }
    {
        const cx<T> q = T(0.25) * b[2];
        kcb.er0 = kcb.er0 + q;
        n.er1 = n.er1 + q;
        if (ax) {
            if (m == 1) {
                jcb.et0 = jcb.et0 + imul(-T(2), q);
                n.et1 = n.et1 + imul(-T(2), q);
            }
            kcb.er0 = kcb.er0 + c.tg * q;
            n.er1 = n.er1 + c.tg * q;
        } else {
            kpb.er0 = kpb.er0 + q;
            n.erl1 = n.erl1 + q;
        }
    }
    if (ax) {
        if (m == 1) kcb.ph0 = kcb.ph0 + imul(T(2) * c.inv_dr, b[3]);
    } else {
        const cx<T> t = T(0.5) * imul(T(m) * c.inv_dr / T(j), b[3]);
        kcb.ph0 = kcb.ph0 + t;
        kpb.ph0 = kpb.ph0 + t;
    }
    {
        const cx<T> q = T(0.5) * b[4];
        jcb.et0 = jcb.et0 + q;
        n.et1 = n.et1 + q;
    }
    {
        const cx<T> s = c.inv_dr * b[5];
        kcb.ph0 = kcb.ph0 + s;
        if (ax) kcb.ph0 = kcb.ph0 - par * s;
        else kpb.ph0 = kpb.ph0 - s;
    }
}
template <typename T>
__device__ __forceinline__ void fac_r_bar(const FacC<T>& c, int j, const cx<T>* b, KRow<T>& kcb, JRow<T>& jcb,
                                          JRow<T>& jnb, NbR<T>& n) {
    {
        const cx<T> q = T(0.125) * b[0];
        jcb.Qp = jcb.Qp + q; n.Qp1 = n.Qp1 + q; jnb.Qp = jnb.Qp + q; n.Qpn1 = n.Qpn1 + q;
    }
    {
        const cx<T> q = T(0.5) * b[1];
        kcb.up = kcb.up + q; n.up1 = n.up1 + q;
    }
    {
        const cx<T> q = T(0.125) * b[2];
        jcb.Qm = jcb.Qm + q; n.Qm1 = n.Qm1 + q; jnb.Qm = jnb.Qm + q; n.Qmn1 = n.Qmn1 + q;
    }
    {
        const cx<T> q = T(0.5) * b[3];
        kcb.wm = kcb.wm + q; n.wm1 = n.wm1 + q;
    }
    {
        const cx<T> q = T(0.5) * b[4];
        jcb.ex = jcb.ex + q; jnb.ex = jnb.ex + q;
    }
    const T irk = T(1) / ((T(j) + T(0.5)) * c.dr);
    kcb.phm = kcb.phm + imul(T(c.m) * irk, b[5]);
}
template <typename T>
__device__ __forceinline__ void fac_t_bar(const FacC<T>& c, int j, const cx<T>* b, KRow<T>& kpb, KRow<T>& kcb,
                                          JRow<T>& jcb, NbT<T>& n) {
    const bool ax = j == 0;
    const int m = c.m;
    const T par = c.par;
    {
        // f0 = fP / 2 with fP = (gP0 + kc.P + gP1 + P1) / 4
        const cx<T> q = T(0.125) * b[0];
        kcb.P = kcb.P + q; n.P1 = n.P1 + q;
        if (ax) {
            if (m == 1) {
                jcb.Qm = jcb.Qm + imul(-T(2), q);
                n.Qm1 = n.Qm1 + imul(-T(2), q);
            }
            kcb.P = kcb.P + c.tg * q; n.P1 = n.P1 + c.tg * q;
        } else {
            kpb.P = kpb.P + q; n.Pl1 = n.Pl1 + q;
        }
    }
    {
        // f4 = -fN / 2
        const cx<T> q = T(-0.125) * b[4];
        kcb.N = kcb.N + q; n.N1 = n.N1 + q;
        if (ax) {
            if (m == 1) {
                jcb.Qp = jcb.Qp + imul(-T(2), q);
                n.Qp1 = n.Qp1 + imul(-T(2), q);
            }
            kcb.N = kcb.N + c.tg * q; n.N1 = n.N1 + c.tg * q;
        } else {
            kpb.N = kpb.N + q; n.Nl1 = n.Nl1 + q;
        }
    }
    {
        const cx<T> q = T(0.25) * b[1];
        kcb.wm = kcb.wm + q; n.wm1 = n.wm1 + q;
        if (ax) {
            kcb.wm = kcb.wm + par * q; n.wm1 = n.wm1 + par * q;
        } else {
            kpb.wm = kpb.wm + q; n.wml1 = n.wml1 + q;
        }
    }
    jcb.ex = jcb.ex + b[2];
    {
        const cx<T> s = c.inv_dr * b[3];
        kcb.phm = kcb.phm + s;
        if (ax) kcb.phm = kcb.phm - par * s;
        else kpb.phm = kpb.phm - s;
    }
    {
        const cx<T> q = T(0.25) * b[5];
        kcb.up = kcb.up + q; n.up1 = n.up1 + q;
        if (ax) {
            kcb.up = kcb.up + par * q; n.up1 = n.up1 + par * q;
        } else {
            kpb.up = kpb.up + q; n.upl1 = n.upl1 + q;
        }
    }
}

// p[o] += v into a new-level plane: an atomic add (it is not waited for, and
// measured faster than a read-add-write whose read has to be held in registers)
template <typename T>
__device__ __forceinline__ void put_new(cx<T>* p, uint32_t o, cx<T> v) {
    cadd((cx<T>*)((char*)p + o), v);
}
// p[o] += v into an old-level plane, which holds zero before this kernel: a
// store where this lane is the point's only writer, else an atomic add
template <typename T>
__device__ __forceinline__ void put_old(cx<T>* p, uint32_t o, cx<T> v, bool atomic) {
    if (atomic) cadd((cx<T>*)((char*)p + o), v);
    else cur::sto(p, o, v);
}

// transposes of cur::load_k / load_j into the plane adjoints
template <typename T>
__device__ __forceinline__ void flush_k(const AxBar<T>& a, uint32_t o, const KRow<T>& b, bool atomic) {
    const cx<T> d = T(0.25) * b.dt0;
    put_old(a.A0b.bx, o, T(0.5) * b.bxn, atomic);
    put_old(a.tapAb, o, d, atomic);
    put_old(a.tamAb, o, d, atomic);
    put_old(a.A0b.trp, o, T(0.5) * (b.er0 + b.P), atomic);
    put_old(a.A0b.trm, o, T(0.5) * (b.er0 + b.N), atomic);
    put_old(a.phiAb, o, b.ph0 + T(0.5) * b.phm, atomic);
    put_new(a.B0b.bx, o, T(0.5) * b.bxn);
    put_new(a.tapBb, o, d + b.up);
    put_new(a.tamBb, o, d + b.wm);
    put_new(a.B0b.trp, o, T(0.5) * b.P);
    put_new(a.B0b.trm, o, T(0.5) * b.N);
    put_new(a.phiBb, o, T(0.5) * b.phm);
}
template <typename T>
__device__ __forceinline__ void flush_j(const AxBar<T>& a, uint32_t o, const JRow<T>& b, bool atomic) {
    put_old(a.A0b.ttp, o, T(0.5) * (b.et0 + b.Qp), atomic);
    put_old(a.A0b.ttm, o, T(0.5) * (b.et0 + b.Qm), atomic);
    put_new(a.B0b.ttp, o, T(0.5) * b.Qp);
    put_new(a.B0b.ttm, o, T(0.5) * b.Qm);
    put_new(a.B0b.ex, o, b.ex);
}

template <typename T, int M>
__global__ void __launch_bounds__(WAVE * M) k_current_bar_march(AxBar<T> a, int rows) {
    const AxionArgs<T>& f = a.f;
    const Geo& g = f.g;
    const int m = threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    // XCD-contiguous runs of tiles, strips fastest (as the forward kernels)
    const int strips = (g.nx + OWN - 1) / OWN;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int strip = tile % strips, chunk = tile / strips;
    const int raw = strip * OWN - 1 + lane;
    // halo lanes wrap with periodic x and are clamped otherwise
    const int i = g.per ? ((raw % g.nx) + g.nx) % g.nx : min(max(raw, 0), g.nx - 1);
    const bool owner = lane >= 1 && lane <= OWN && raw < g.nx;
    const bool has1 = g.per || i + 1 < g.nx;
    // cells computed here: inside the domain, not the dead last cell, and for a
    // clamped halo lane not a copy of the first cell
    const bool live = (g.per || i < g.nx - 1) && (g.per || raw >= 0);
    const int r0 = chunk * rows;
    const int r1 = min(g.nr, r0 + rows);
    const T dr = T(g.dr);
    const FacC<T> fc{m, parity<T>(m), tghost<T>(m), dr, T(1) / dr, f.bx0, f.br1, f.bt1};
    const T sj = T(f.s_j);
    const cx<T> zc = zero<T>();

    // two exchange buffers used alternately by the three phases of a row, so
    // one barrier per phase keeps writers behind the last readers
    __shared__ cx<T> sm[2][7][M][WAVE];
    int ph = 0;
    double dsj = 0.0;

    // one phase: exchange the own factors f and own j_a adjoint jb, then the
    // adjoints fb of the own factors (and the own-mode output for dL/ds_j,
    // counted once per cell: on the lane that owns its column)
    auto phase = [&](const cx<T>* fo, cx<T> jbo, bool calc, cx<T>* fb) {
        if (calc) {
#pragma unroll
            for (int q = 0; q < 6; ++q) sm[ph][q][m][lane] = fo[q];
            sm[ph][6][m][lane] = jbo;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 6; ++q) fb[q] = zc;
        if (calc) {
            cx<T> Ob[M];
#pragma unroll
            for (int k = 0; k < M; ++k) Ob[k] = sj * sm[ph][6][k][lane];
            cx<T> out = zc;
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                cx<T> A[M], B[M];
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    A[k] = sm[ph][2 * p][k][lane];
                    B[k] = sm[ph][2 * p + 1][k][lane];
                }
                const T sgn = p == 1 ? T(-1) : T(1);
                conv_bar_one<T, M>(A, B, Ob, sgn, m, fb[2 * p], fb[2 * p + 1]);
                if (a.dLds) conv_one<T, M>(A, B, m, out, sgn);
            }
            if (owner) dsj += double(jbo.re) * double(out.re) + double(jbo.im) * double(out.im);
        }
        ph ^= 1;
    };

    KRow<T> kp = r0 >= 1 ? cur::load_k(f, cur::eoff<T>(g, m, r0 - 1, i)) : cur::zero_k<T>();
    JRow<T> jc = cur::load_j(f, cur::eoff<T>(g, m, r0, i));
    KRow<T> kpb = cur::zero_k<T>();   // adjoint of K row j-1 (its share from row j-1)
    JRow<T> jcb = cur::zero_j<T>();   // adjoint of J row j (its share from row j-1)
    for (int j = r0; j < r1; ++j) {
        const uint32_t o = cur::eoff<T>(g, m, j, i);
        const KRow<T> kc = cur::load_k(f, o);
        const JRow<T> jn = cur::load_j(f, cur::eoff<T>(g, m, j + 1, i));
        const cx<T> jxb = cur::ldo(a.jaxb, o), jrb = cur::ldo(a.jarb, o), jtb = cur::ldo(a.jatb, o);
        const uint32_t ok = cur::eoff<T>(g, m, j >= 1 ? j - 1 : 0, i);
        KRow<T> kcb = cur::zero_k<T>();
        JRow<T> jnb = cur::zero_j<T>();
        {
            // j_a,theta
            const NbT<T> nt = cur::nb_t(kp, kc, jc, has1);
            cx<T> fo[6], fb[6];
            if (live) cur::fac_t(fc, j, kp, kc, jc, nt, fo);
            phase(fo, jtb, live, fb);
            NbT<T> nb{zc, zc, zc, zc, zc, zc, zc, zc, zc, zc};
            if (live) fac_t_bar(fc, j, fb, kpb, kcb, jcb, nb);
            prev_add(kcb.P, nb.P1); prev_add(kcb.N, nb.N1); prev_add(kcb.up, nb.up1); prev_add(kcb.wm, nb.wm1);
            prev_add(kpb.P, nb.Pl1); prev_add(kpb.N, nb.Nl1); prev_add(kpb.up, nb.upl1); prev_add(kpb.wm, nb.wml1);
            prev_add(jcb.Qp, nb.Qp1); prev_add(jcb.Qm, nb.Qm1);
        }
        {
            // j_a,x
            const NbX<T> nx = cur::nb_x(kp, kc, jc, has1);
            cx<T> fo[6], fb[6];
            if (live) cur::fac_x(fc, j, kp, kc, jc, nx, fo);
            phase(fo, jxb, live, fb);
            NbX<T> nb{zc, zc, zc, zc, zc};
            if (live) fac_x_bar(fc, j, fb, kpb, kcb, jcb, nb);
            prev_add(kcb.dt0, nb.dt1); prev_add(kcb.er0, nb.er1); prev_add(jcb.et0, nb.et1);
            prev_add(kpb.dt0, nb.dtl1); prev_add(kpb.er0, nb.erl1);
        }
        // K row j-1 is complete (only the theta and x factors read it), except
        // for the row shared with the chunk below
        if (owner && j >= 1) flush_k(a, ok, kpb, j == r0);
        {
            // j_a,r
            const NbR<T> nr = cur::nb_r(kc, jc, jn, has1);
            cx<T> fo[6], fb[6];
            if (live) cur::fac_r(fc, j, kc, jc, jn, nr, fo);
            phase(fo, jrb, live, fb);
            NbR<T> nb{zc, zc, zc, zc, zc, zc};
            if (live) fac_r_bar(fc, j, fb, kcb, jcb, jnb, nb);
            prev_add(jcb.Qp, nb.Qp1); prev_add(jcb.Qm, nb.Qm1); prev_add(jnb.Qp, nb.Qpn1);
            prev_add(jnb.Qm, nb.Qmn1); prev_add(kcb.up, nb.up1); prev_add(kcb.wm, nb.wm1);
        }
        // J row j is complete, except for the row shared with the chunk below
        if (owner) flush_j(a, o, jcb, j == r0 && r0 > 0);
        kp = kc;
        jc = jn;
        kpb = kcb;
        jcb = jnb;
    }
    if (owner) {
        // K row r1-1 and J row r1: complete in the last chunk, shared otherwise
        const uint32_t ok = cur::eoff<T>(g, m, r1 - 1, i), oj = cur::eoff<T>(g, m, r1, i);
        flush_k(a, ok, kpb, r1 != g.nr);
        flush_j(a, oj, jcb, r1 != g.nr);
    }
    if (a.dLds) {
        // one atomic per wave
#pragma unroll
        for (int s = WAVE / 2; s > 0; s >>= 1) dsj += __shfl_xor(dsj, s, WAVE);
        if (lane == 0 && dsj != 0.0) atomicAdd(a.dLds + 1, dsj);
    }
}

}  // namespace curb

}  // namespace adj

// ---------------------------------------------------------------------------
// host-side adjoint of one staged step
// ---------------------------------------------------------------------------
template <typename T>
static adj::SetBar<T> setbar(cx<T>* const* P, int s) {
    const int b = 9 * s;
    return adj::SetBar<T>{P[b + 0], P[b + 1], P[b + 2], P[b + 3], P[b + 4], P[b + 5], P[b + 6], P[b + 7], P[b + 8]};
}

template <typename T>
static adj::StageBar<T> stage_bar(const StepPlan<T>& p, cx<T>* const* Ab, cx<T>* const* Bb, cx<T>* const* jab, int s) {
    StageArgs<T> f = p.set_args(s);
    adj::StageBar<T> a;
    a.g = p.g;
    a.A = f.A;
    a.B = f.B;
    a.Ab = setbar(Ab, s);
    a.Bb = setbar(Bb, s);
    a.jx_addb = s ? jab[0] : nullptr;
    a.jr_addb = s ? jab[1] : nullptr;
    a.jt_addb = s ? jab[2] : nullptr;
    a.plasma = p.plasma;
    a.wp2 = p.wp2;
    return a;
}

// cell rows per workgroup of the marched current adjoint
constexpr int kCurBarRows = 6;

template <typename T, int M>
static void launch_axion_bar(adj::AxBar<T>& a, bool arem, bool march, hipStream_t s) {
    const Geo& g = a.f.g;
    dim3 blk(64, 4);
    dim3 grdK((g.nx + 63) / 64, (g.nr + 3) / 4);
    if (arem) {
        // the march addresses a plane through 32-bit byte offsets
        const size_t plane = size_t(g.M) * size_t(g.nr + 1) * size_t(g.ld) * sizeof(cx<T>);
        if (march && plane < (size_t(1) << 32)) {
            const int rows = kCurBarRows;
            const int strips = (g.nx + adj::curb::OWN - 1) / adj::curb::OWN;
            const int chunks = (g.nr + rows - 1) / rows;
            hipLaunchKernelGGL((adj::curb::k_current_bar_march<T, M>), dim3(strips * chunks),
                               dim3(adj::curb::WAVE * M), 0, s, a, rows);
        } else {
            hipLaunchKernelGGL((adj::k_axion_current_bar<T, M>), grdK, blk, 0, s, a);
        }
    }
    hipLaunchKernelGGL(adj::k_axion_phi_bar<T>, grdK, blk, 0, s, a);
    hipLaunchKernelGGL((adj::k_axion_ta_bar<T, M>), grdK, blk, 0, s, a);
}

template <typename T>
hipError_t adjoint_step(const StepPlan<T>& p, cx<T>* const* Ab, cx<T>* const* Bb, cx<T>* const* jab, double* dLds,
                        bool march, hipStream_t s) {
    const Geo& g = p.g;
    dim3 blk(64, 4);
    dim3 grdJ((g.nx + 63) / 64, (g.nr + 1 + 3) / 4);
    dim3 grdG((g.nx + 63) / 64, g.M);          // exterior ghost row: one wave per 64 columns and mode
    dim3 grdL((g.nx + adj::kLongOwn - 1) / adj::kLongOwn, (g.nr + 1 + 3) / 4);
    if (p.axion && p.arem) {
        adj::StageBar<T> a1 = stage_bar(p, Ab, Bb, jab, 1);
        hipLaunchKernelGGL(adj::k_ghost_bth_bar<T>, grdG, dim3(64), 0, s, a1);
        hipLaunchKernelGGL(adj::k_transverse_bar<T>, grdJ, blk, 0, s, a1);
        hipLaunchKernelGGL(adj::k_longitudinal_bar<T>, grdL, blk, 0, s, a1);
        if (g.open_r) hipLaunchKernelGGL(adj::k_longitudinal_ghost_bar<T>, grdG, dim3(64), 0, s, a1);
    }
    if (p.axion) {
        adj::AxBar<T> ax;
        ax.f = p.axion_args();
        ax.A0b = setbar(Ab, 0);
        ax.B0b = setbar(Bb, 0);
        ax.phiAb = Ab[18]; ax.tapAb = Ab[19]; ax.tamAb = Ab[20];
        ax.phiBb = Bb[18]; ax.tapBb = Bb[19]; ax.tamBb = Bb[20];
        ax.jaxb = jab[0]; ax.jarb = jab[1]; ax.jatb = jab[2];
        ax.dLds = dLds;
        switch (g.M) {
#define QDS_AXB(MM) case MM: launch_axion_bar<T, MM>(ax, p.arem, march, s); break;
            QDS_AXB(1) QDS_AXB(2) QDS_AXB(3) QDS_AXB(4)
#undef QDS_AXB
            default: return hipErrorInvalidValue;
        }
    }
    adj::StageBar<T> a0 = stage_bar(p, Ab, Bb, jab, 0);
    hipLaunchKernelGGL(adj::k_ghost_bth_bar<T>, grdG, dim3(64), 0, s, a0);
    hipLaunchKernelGGL(adj::k_transverse_bar<T>, grdJ, blk, 0, s, a0);
    hipLaunchKernelGGL(adj::k_longitudinal_bar<T>, grdL, blk, 0, s, a0);
    if (g.open_r) hipLaunchKernelGGL(adj::k_longitudinal_ghost_bar<T>, grdG, dim3(64), 0, s, a0);
    return hipGetLastError();
}

template hipError_t adjoint_step<double>(const StepPlan<double>&, cx<double>* const*, cx<double>* const*,
                                         cx<double>* const*, double*, bool, hipStream_t);
template hipError_t adjoint_step<float>(const StepPlan<float>&, cx<float>* const*, cx<float>* const*,
                                        cx<float>* const*, double*, bool, hipStream_t);

}  // namespace qds

namespace qds {
namespace adj {

// Loss: energy of one mode of one set over the columns [x0, x1):
//   L = w h dr [ sum_K r_{k+1/2} (|T_r^+|^2 + |T_r^-|^2)/4 + sum_J r'_j (|T_th^+|^2 + |T_th^-|^2)/4
//              + sum_J r'_j |E_x|^2/2 + sum_K r_{k+1/2} |B_x|^2/2 ]
// with w = 2 pi (mode 0) or pi, r'_0 = dr/8, r'_j = j dr.  Writes dL/du = 2 c u
// into the adjoint buffer and adds L to *loss.
template <typename T>
__global__ void __launch_bounds__(256) k_loss_seed(SetPtr<T> u, SetBar<T> ub, Geo g, int md, int x0, int x1, double* loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double acc = 0.0;
    if (i >= x0 && i < x1 && i < g.nx && j <= g.nr) {
        const double pi = 3.141592653589793;
        const double w = (md == 0 ? 2.0 * pi : pi) * g.h * g.dr;
        const double rk = (j + 0.5) * g.dr;
        const double rj = j == 0 ? g.dr / 8.0 : j * g.dr;
        auto one = [&](const cx<T>* p, cx<T>* pb, double c) {
            const size_t e = g.at(md, j, i);
            cx<T> v = ld(p + e);
            acc += c * (double(v.re) * v.re + double(v.im) * v.im);
            st(pb + e, T(2.0 * c) * v);
        };
        if (j < g.nr) {
            one(u.trp, ub.trp, 0.25 * w * rk);
            one(u.trm, ub.trm, 0.25 * w * rk);
            one(u.bx, ub.bx, 0.5 * w * rk);
        }
        one(u.ttp, ub.ttp, 0.25 * w * rj);
        one(u.ttm, ub.ttm, 0.25 * w * rj);
        one(u.ex, ub.ex, 0.5 * w * rj);
    }
    block_sum_add(acc, loss);
}

// real inner product sum Re(conj(a) b) over n complex elements
template <typename T>
__global__ void __launch_bounds__(256) k_dot(const cx<T>* a, const cx<T>* b, size_t n, double* out) {
    double acc = 0.0;
    for (size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += size_t(gridDim.x) * blockDim.x) {
        cx<T> x = ld(a + q), y = ld(b + q);
        acc += double(x.re) * y.re + double(x.im) * y.im;
    }
    block_sum_add(acc, out);
}

}  // namespace adj

template <typename T>
hipError_t loss_seed(cx<T>* const* U, cx<T>* const* Ub, const Geo& g, int set, int md, int x0, int x1, double* loss,
                     hipStream_t s) {
    const int b = 9 * set;
    SetPtr<T> u{U[b + 0], U[b + 1], U[b + 2], U[b + 3], U[b + 4], U[b + 5], U[b + 6], U[b + 7], U[b + 8]};
    adj::SetBar<T> ub{Ub[b + 0], Ub[b + 1], Ub[b + 2], Ub[b + 3], Ub[b + 4], Ub[b + 5], Ub[b + 6], Ub[b + 7], Ub[b + 8]};
    dim3 blk(64, 4);
    dim3 grd((g.nx + 63) / 64, (g.nr + 1 + 3) / 4);
    hipLaunchKernelGGL(adj::k_loss_seed<T>, grd, blk, 0, s, u, ub, g, md, x0, x1, loss);
    return hipGetLastError();
}

template <typename T>
hipError_t dot(const void* a, const void* b, size_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(adj::k_dot<T>, dim3(1024), dim3(256), 0, s, static_cast<const cx<T>*>(a),
                       static_cast<const cx<T>*>(b), n, out);
    return hipGetLastError();
}

template hipError_t loss_seed<double>(cx<double>* const*, cx<double>* const*, const Geo&, int, int, int, int, double*,
                                      hipStream_t);
template hipError_t loss_seed<float>(cx<float>* const*, cx<float>* const*, const Geo&, int, int, int, int, double*,
                                     hipStream_t);
template hipError_t dot<double>(const void*, const void*, size_t, double*, hipStream_t);
template hipError_t dot<float>(const void*, const void*, size_t, double*, hipStream_t);

}  // namespace qds
