// Fused single-pass QDS step for gfx950.
//
// Layout of the work: a workgroup of kernel A is one wavefront per mode; wave
// w advances mode m = w of one strip of 64 half-x cells (lanes; 61 owned, lane
// 0 a left halo, lanes 62-63 a right halo) over one chunk of radial rows.
// Each lane marches the rows in increasing r keeping a sliding window of rows
// in registers, so every state plane is read once and written once per step;
// the values of column i+1 come from the next lane by a DPP shift and the
// neighbouring cells' new transport values from lane shuffles.  The azimuthal
// mode convolution of the axion source exchanges its per-mode factors through
// LDS between the waves of the workgroup.  Kernel B is the same march for one
// set, one wave per (strip, chunk, mode).
//
// Kernel A advances the background set and forms the axion source S_a.  With
// the regenerated set (and no moving window) it leaves S_a in a scratch plane
// and the marched kernel of qds_current.hip advances the axion (Klein-Gordon
// transport, phi) together with the axion current at the source points;
// otherwise kernel A advances the axion itself.  Kernel B advances the
// regenerated set with the axion current.  A prescribed drive is evaluated
// per step into a plane of its own (k_drive_plane) that the background set
// reads as an extra j_x of mode 0.  They compute exactly the quantities of
// the staged kernels.
//
// Temporal blocking: the two-step march (em2_body) advances one set through
// two steps in one pass, its first step's rows handed to a second wave
// through an LDS ring, so the set's planes are read and written once per two
// steps (the regenerated set in pairs of steps, or the background set of an
// electromagnetic-only run, also with the moving window and the drive).
// fused_a2_body does the same for the background set with the axion source of
// both steps (2M waves per workgroup; an option, measured slower).
#include "qds_current_rows.hpp"

namespace qds {
namespace fused {

constexpr int WAVE = 64;
constexpr int OWN = kFusedOwn;   // owned cells per wave (lane 0 and lanes 62-63 are halos)

// Byte offset of element (m, row, c) inside a plane.  A plane is below 4 GiB
// (checked when the handle is created), so one 32-bit per-lane offset serves
// every plane: the loads take the uniform plane base in scalar registers.
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

template <typename T>
struct XAcc {
    // column helpers for one lane: H cell i, integer columns i and i+1
    int nr1, ld;     // rows per mode and row pitch of a plane
    int i;
    int i1;          // column of x_{i+1} (wrapped if periodic, -1 outside)
    int ir;          // destination column of right movers (i+1), -1 outside
    __device__ __forceinline__ uint32_t ro(int m, int row) const {
        return uint32_t(m * nr1 + row) * uint32_t(ld) * uint32_t(sizeof(cx<T>));
    }
    __device__ __forceinline__ cx<T> L(const cx<T>* p, int m, int row) const {
        return ldo(p, ro(m, row) + uint32_t(i) * uint32_t(sizeof(cx<T>)));
    }
    __device__ __forceinline__ cx<T> R(const cx<T>* p, int m, int row) const {
        return i1 >= 0 ? ldo(p, ro(m, row) + uint32_t(i1) * uint32_t(sizeof(cx<T>))) : zero<T>();
    }
    // column i+1 from the next lane's column-i value (all lanes active)
    __device__ __forceinline__ cx<T> Rn(cx<T> a) const {
        const cx<T> b = next_lane(a);
        return i1 >= 0 ? b : zero<T>();
    }
};

template <typename T>
__device__ __forceinline__ cx<T> shfl_up1(cx<T> v) {
    return cx<T>{__shfl_up(v.re, 1, WAVE), __shfl_up(v.im, 1, WAVE)};
}
template <typename T>
__device__ __forceinline__ cx<T> shfl_dn1(cx<T> v) {
    return cx<T>{__shfl_down(v.re, 1, WAVE), __shfl_down(v.im, 1, WAVE)};
}

// Prescribed j_x^(0) of step n + z at (x_{i+1/2}, r_j, t^{n+z}), lab column
// i + w + z dw, into the mode-0 rows of plane z of a launch (row pitch g.ld;
// z = blockIdx.z, one or two planes: a pair of steps fills both in one launch).
// A thread holds one column over kDriveRows rows: the x Gaussian is evaluated
// once per thread and the r Gaussian once per row of the workgroup, so a point
// costs its normal variate only (the same expressions as one evaluation per
// point, hence the same bits).  The marching kernels read it as an extra
// current and carry none of its exponentials and variates in their registers.
constexpr int kDriveRows = 8;

template <typename T>
__global__ void __launch_bounds__(256) k_drive_plane(Drive d, Geo g, cx<T>* out0, cx<T>* out1, int64_t n, int64_t w,
                                                     int64_t dw) {
    const int z = blockIdx.z;
    const int64_t nz = n + z, wz = w + z * dw;
    cx<T>* const out = z ? out1 : out0;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j0 = blockIdx.y * kDriveRows;
    const int j1 = min(g.nr + 1, j0 + kDriveRows);
    __shared__ double grs[kDriveRows];
    if (threadIdx.x < kDriveRows) {
        const double r = double(j0 + int(threadIdx.x)) * g.dr;
        const double ar = r - d.r0;
        grs[threadIdx.x] = exp(-ar * ar / (2.0 * d.sr * d.sr));
    }
    __syncthreads();
    if (i >= g.nx) return;
    const double x = (double(i) + 0.5 + double(wz)) * g.h;
    const double t = double(nz) * g.h;
    const double ax = x - d.x0 - d.v * t;
    const double gx = exp(-ax * ax / (2.0 * d.sx * d.sx));
    for (int j = j0; j < j1; ++j) {
        const double gr = grs[j - j0];
        const uint64_t c = (uint64_t(nz) << 32) | (uint64_t(int64_t(i) + wz) << 12) | uint64_t(j);
        const double v = d.amp * gr * gx * (1.0 + d.noise * normal_ctr(d.seed, c));
        st(out + size_t(j) * size_t(g.ld) + size_t(i), cx<T>{T(v), T(0)});
    }
}

// Output addressing: with the moving window every write lands one column to
// the left and the last column is zero-filled by the owner of the last cell.
struct Out {
    int shift;
    int nx;
    __device__ __forceinline__ int col(int c) const { return c - shift; }
};

// ---------------------------------------------------------------------------
// the electromagnetic part of a set, marched in r
// ---------------------------------------------------------------------------
template <typename T>
struct EmWin {
    // T_r^+- at K rows j (slot 0) and j+1 (slot 1), column i (the values of
    // column i+1 are the next lane's, see EmB)
    cx<T> rpa[2], rma[2];
    // T_theta^+- at J rows j (slot 0) and j+1 (slot 1)
    cx<T> tpa[2], tma[2];
    cx<T> ex0[2];      // E_x^{n-1/2} at J = j, j+1
    cx<T> ex1[3];      // E_x^{n+1/2} at J = j-1, j, j+1
    cx<T> bx0[2];      // B_x^{n-1/2} at K = j, j+1
    cx<T> bx1[2];      // B_x^{n+1/2} at K = j-1, j
    cx<T> bx1g;        // exterior ghost B_x^{n+1/2}
    cx<T> jx_n1;       // total j_x at (x_{i+1/2}, r_{j+1}, t^n) (used for E_x(J=j+1))
    cx<T> jx_nr;       // total j_x at row nr (for the ghost B_theta)
    cx<T> pjx, pjxa;   // plasma j_x^{n-1} and extra j_x on J = j+1 (loaded ahead)
    // new transverse values after the transport of this step (both columns)
    cx<T> n_rpa, n_rpb, n_rma, n_rmb;   // T_r^{n+1} at K = j
    cx<T> n_tpa, n_tpb, n_tma, n_tmb;   // T_theta^{n+1} at J = j
};


// Column i+1 of the window's transverse values for one march step, taken
// from the next lane (built in uniform control flow at the top of the step).
template <typename T>
struct EmB {
    cx<T> rpb[2], rmb[2], tpb[2], tmb[2];
};

template <typename T>
struct Ctx {
    Geo g;
    int m;           // mode of this wave
    int lane;
    int i;           // H cell
    bool live;       // H cell inside the domain
    bool owner;      // lane owns cell i
    XAcc<T> x;
    Out o;
    T h, dr;
    T inv_dr, inv_2dr;   // 1/dr, 1/(2 dr)
    T kap, cR;           // outer-ghost centring: (dr - h)/(dr + h), 2 h dr/(dr + h)
    T inv_2h;            // 1/(2 h)
    T wp2h;
    int plasma;
    // the first step of the two-step march with the moving window: this
    // lane's column is the one the window brings in, so what it puts in the
    // ring is the zero-filled state
    bool rzero;
    int gr0, gr1;    // IO_RING_G: rows whose field values also go to the output planes
};

// reciprocal radii of one march step: 1/r_{j+1}, 1/r_{j+1/2}, 1/r_j (0 on the axis)
template <typename T>
struct RowInv {
    T irJ1, irK, irJ;
};
template <typename T>
__device__ __forceinline__ RowInv<T> row_inv(const Ctx<T>& c, int j) {
    RowInv<T> q;
    q.irJ1 = T(1) / (T(j + 1) * c.dr);
    q.irK = T(1) / ((T(j) + T(0.5)) * c.dr);
    q.irJ = j > 0 ? T(1) / (T(j) * c.dr) : T(0);
    return q;
}

// The values of row k = j + 1 that iteration j of the march consumes, loaded
// one iteration ahead so that their latency overlaps the arithmetic of the
// previous row (T_r on K = k or the ghost B_theta, T_theta, E_x^{n-1/2} and
// B_x^{n-1/2} on J/K = k, the plasma j_x and the extra j_x on J = k).
template <typename T>
struct EmPf {
    cx<T> rpa, rpb, rma, rmb, tpa, tpb, tma, tmb, ex0, bx0, jx, jxa;
};

template <typename T>
__device__ __forceinline__ EmPf<T> em_fetch(const Ctx<T>& c, const SetP<T>& s, int k) {
    const int m = c.m;
    EmPf<T> p;
    p.rpa = p.rpb = p.rma = p.rmb = p.tpa = p.tpb = p.tma = p.tmb = zero<T>();
    p.ex0 = p.bx0 = p.jx = p.jxa = zero<T>();
    if (k < 0) return p;
    if (k < c.g.nr) {
        p.rpa = c.x.L(s.trp, m, k);
        p.rma = c.x.L(s.trm, m, k);
    } else if (k == c.g.nr) {
        // exterior ghost row: B_theta stored in the T_r^+ plane, expressed as
        // T_r^+ = B_theta, T_r^- = -B_theta so that (T+ - T-)/2 = B_theta
        cx<T> a = c.x.L(s.trp, m, k);
        p.rpa = a; p.rma = -a;
    }
    if (k <= c.g.nr) {
        p.tpa = c.x.L(s.ttp, m, k);
        p.tma = c.x.L(s.ttm, m, k);
        p.ex0 = c.x.L(s.ex, m, k);
        p.bx0 = c.x.L(s.bx, m, k);
        if (c.plasma) p.jx = c.x.L(s.jx, m, k);
        if (s.jxa && c.live && (!s.jxa_m0 || m == 0)) p.jxa = c.x.L(s.jxa, m, k);
    }
    return p;
}

// moves a fetched row into slot 1
template <typename T>
__device__ __forceinline__ void em_take(const Ctx<T>& c, EmWin<T>& W, const EmPf<T>& p, int k, int nr) {
    if (k > nr) return;
    W.rpa[1] = p.rpa; W.rma[1] = p.rma;
    W.tpa[1] = p.tpa; W.tma[1] = p.tma;
    W.ex0[1] = p.ex0;
    W.bx0[1] = p.bx0;
    W.pjx = p.jx;
    W.pjxa = p.jxa;
}

// The currents of row j that iteration j of the march reads at column i
// (plasma j_r, j_theta; the extra j_r, j_theta of the regenerated set), issued
// together at the top of the iteration; column i+1 comes from the next lane.
template <typename T>
struct EmRowX {
    cx<T> jr, jt, jra, jta;
};
template <typename T>
__device__ __forceinline__ EmRowX<T> em_fetch_x(const Ctx<T>& c, const SetP<T>& s, int j) {
    EmRowX<T> x;
    x.jr = x.jt = x.jra = x.jta = zero<T>();
    if (j < 0) return x;
    if (c.plasma) {
        if (j < c.g.nr) x.jr = c.x.L(s.jr, c.m, j);
        x.jt = c.x.L(s.jt, c.m, j);
    }
    if (s.jra && j < c.g.nr) x.jra = c.x.L(s.jra, c.m, j);
    if (s.jta) x.jta = c.x.L(s.jta, c.m, j);
    return x;
}

// column i+1 of both window slots from the next lane (every lane active)
template <typename T>
__device__ __forceinline__ EmB<T> em_bvals(const Ctx<T>& c, const EmWin<T>& W) {
    EmB<T> B;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        B.rpb[q] = c.x.Rn(W.rpa[q]);
        B.rmb[q] = c.x.Rn(W.rma[q]);
        B.tpb[q] = c.x.Rn(W.tpa[q]);
        B.tmb[q] = c.x.Rn(W.tma[q]);
    }
    return B;
}

// Where a march writes the new state.  IO_GLOBAL: the owner lanes store the
// rows [r0, r1) of their columns to the output planes.  IO_RING (the first
// step of the two-step march): every lane puts the values of its own column,
// for the rows [r0, r1), into the workgroup's LDS ring, from which the second
// step reads them in place of the state planes.  IO_FROM_RING (that second
// step): global stores as IO_GLOBAL, and the old plasma j_theta that the
// exterior ghost reads comes from the ring.
// IO_RING_G (the first step of the background set's two-step march with the
// axion source): the ring as IO_RING and, for the rows [c.gr0, c.gr1), the
// field planes (T^+-, E_x, B_x: what the axion kernel reads) to the output
// planes as IO_GLOBAL; the currents go to the ring only.
enum { IO_GLOBAL = 0, IO_RING = 1, IO_FROM_RING = 2, IO_RING_G = 3 };

// The LDS ring of the two-step march: the 9 planes of one set (T_r^+-,
// T_theta^+-, E_x, B_x, j_x, j_r, j_theta) for 4 consecutive rows (row k in
// slot k mod 4) of the 64 lanes of a strip, lane-contiguous.
enum { RG_TRP = 0, RG_TRM, RG_TTP, RG_TTM, RG_EX, RG_BX, RG_JX, RG_JR, RG_JT, RG_N };
constexpr int RING_ROWS = 4;
template <typename T>
__device__ __forceinline__ cx<T>* rg(cx<T>* ring, int plane, int row, int lane) {
    return ring + (plane * RING_ROWS + (row & (RING_ROWS - 1))) * WAVE + lane;
}
// one value of the lane's own column into the ring
template <typename T>
__device__ __forceinline__ void rput(const Ctx<T>& c, cx<T>* ring, int plane, int row, cx<T> v) {
    *rg(ring, plane, row, c.lane) = c.rzero ? zero<T>() : v;
}

// total j_x at (x_{i+1/2}, r_row, t^n): plasma j_x^n + extra (the axion
// current, or the prescribed drive)
template <typename T, int IO = IO_GLOBAL>
__device__ __forceinline__ cx<T> em_jx(const Ctx<T>& c, const SetP<T>& s, int row, cx<T> ex0, bool write,
                                      cx<T> jx_old, cx<T> jxa, cx<T>* ring = nullptr) {
    cx<T> v = zero<T>();
    if (!c.live) {
        // the dead last cell: its plasma current still advances (it enters no field)
        if constexpr (IO == IO_RING) {
            if (c.plasma && write) rput(c, ring, RG_JX, row, jx_old + c.wp2h * ex0);
        } else {
            if (c.plasma && write && c.owner && c.o.col(c.i) >= 0)
                sto(s.ojx, eoff<T>(c.g, c.m, row, c.o.col(c.i)), jx_old + c.wp2h * ex0);
        }
        return v;
    }
    if (c.plasma) {
        cx<T> jn = jx_old + c.wp2h * ex0;
        if constexpr (IO == IO_RING) {
            if (write) rput(c, ring, RG_JX, row, jn);
        } else {
            if (write && c.owner && c.o.col(c.i) >= 0) sto(s.ojx, eoff<T>(c.g, c.m, row, c.o.col(c.i)), jn);
        }
        v = jn;
    }
    if (s.jxa) v = v + jxa;
    return v;
}

// Row k of the first step's results, from the ring, for the second step of
// the two-step march (the values em_fetch reads from the state planes), with
// the second step's extra j_x of row k, loaded a row ahead (em_xa).
template <typename T>
__device__ __forceinline__ EmPf<T> em_fetch_ring(const Ctx<T>& c, cx<T>* ring, int k, cx<T> jxa) {
    const int l = c.lane;
    EmPf<T> p;
    p.rpa = p.rpb = p.rma = p.rmb = p.tpa = p.tpb = p.tma = p.tmb = zero<T>();
    p.ex0 = p.bx0 = p.jx = p.jxa = zero<T>();
    if (k < 0) return p;
    if (k < c.g.nr) {
        p.rpa = *rg(ring, RG_TRP, k, l);
        p.rma = *rg(ring, RG_TRM, k, l);
    } else if (k == c.g.nr) {
        const cx<T> a = *rg(ring, RG_TRP, k, l);   // the exterior ghost B_theta
        p.rpa = a; p.rma = -a;
    }
    if (k <= c.g.nr) {
        p.tpa = *rg(ring, RG_TTP, k, l);
        p.tma = *rg(ring, RG_TTM, k, l);
        p.ex0 = *rg(ring, RG_EX, k, l);
        p.bx0 = *rg(ring, RG_BX, k, l);
        if (c.plasma) p.jx = *rg(ring, RG_JX, k, l);
        p.jxa = jxa;
    }
    return p;
}
template <typename T>
__device__ __forceinline__ EmRowX<T> em_fetch_x_ring(const Ctx<T>& c, cx<T>* ring, int j, const EmRowX<T>& ext) {
    EmRowX<T> x;
    x.jr = x.jt = x.jra = x.jta = zero<T>();
    if (j < 0) return x;
    if (c.plasma) {
        if (j < c.g.nr) x.jr = *rg(ring, RG_JR, j, c.lane);
        x.jt = *rg(ring, RG_JT, j, c.lane);
    }
    x.jra = ext.jra;
    x.jta = ext.jta;
    return x;
}
// The extra currents that the march reads from their planes (not from the
// ring): j_x of row k, and j_r, j_theta of row j (zero where em_fetch and
// em_fetch_x read none).
template <typename T>
__device__ __forceinline__ cx<T> em_xa(const Ctx<T>& c, const SetP<T>& s, int k) {
    if (k < 0 || k > c.g.nr || !s.jxa || !c.live || (s.jxa_m0 && c.m != 0)) return zero<T>();
    return c.x.L(s.jxa, c.m, k);
}
template <typename T>
__device__ __forceinline__ EmRowX<T> em_xrt(const Ctx<T>& c, const SetP<T>& s, int j) {
    EmRowX<T> x;
    x.jr = x.jt = x.jra = x.jta = zero<T>();
    if (j < 0) return x;
    if (s.jra && j < c.g.nr) x.jra = c.x.L(s.jra, c.m, j);
    if (s.jta && j <= c.g.nr) x.jta = c.x.L(s.jta, c.m, j);
    return x;
}

// E_x^{n+1/2} at J = j+1 from the window (Eqs. Ex_update, Gammax_explicit, axis_Ex)
template <typename T>
__device__ __forceinline__ cx<T> em_ex_new(const Ctx<T>& c, const EmWin<T>& W, const EmB<T>& B, int jj, cx<T> jx,
                                          T irj) {
    const T h = c.h;
    const int m = c.m;
    if (!c.live || (!c.g.open_r && jj == c.g.nr)) return zero<T>();
    if (jj == 0) {
        if (m != 0) return zero<T>();
        cx<T> b = T(0.25) * ((W.rpa[1] - W.rma[1]) + (B.rpb[1] - B.rmb[1]));
        return W.ex0[1] + h * ((T(4) * c.inv_dr) * b - jx);
    }
    cx<T> lo0 = T(0.5) * (W.rpa[0] - W.rma[0]), lo1 = T(0.5) * (B.rpb[0] - B.rmb[0]);
    cx<T> hi0 = T(0.5) * (W.rpa[1] - W.rma[1]), hi1 = T(0.5) * (B.rpb[1] - B.rmb[1]);
    cx<T> bavg = T(0.25) * (lo0 + hi0 + lo1 + hi1);
    cx<T> db = c.inv_2dr * ((hi0 + hi1) - (lo0 + lo1));
    cx<T> bravg = T(0.25) * ((W.tpa[1] - W.tma[1]) + (B.tpb[1] - B.tmb[1]));
    cx<T> gx = irj * bavg + db + imul(T(m) * irj, bravg) - jx;
    return W.ex0[1] + h * gx;
}

// B_x^{n+1/2} at K = j (Eqs. Ex_update, Phix_explicit)
template <typename T>
__device__ __forceinline__ cx<T> em_bx_new(const Ctx<T>& c, const EmWin<T>& W, const EmB<T>& B, T irk) {
    if (!c.live) return zero<T>();
    const T h = c.h;
    cx<T> lo0 = T(0.5) * (W.tpa[0] + W.tma[0]), lo1 = T(0.5) * (B.tpb[0] + B.tmb[0]);
    cx<T> hi0 = T(0.5) * (W.tpa[1] + W.tma[1]), hi1 = T(0.5) * (B.tpb[1] + B.tmb[1]);
    cx<T> eavg = T(0.25) * (lo0 + hi0 + lo1 + hi1);
    cx<T> de = c.inv_2dr * ((hi0 + hi1) - (lo0 + lo1));
    cx<T> eravg = T(0.25) * ((W.rpa[0] + W.rma[0]) + (B.rpb[0] + B.rmb[0]));
    cx<T> fx = -(irk * eavg + de) - imul(T(c.m) * irk, eravg);
    return W.bx0[0] + h * fx;
}

// plasma j_theta at (x_{i+1/2}, r_j, t^{n+1/2}) from the window slot s and the
// old plasma j_theta at columns i (jti) and i+1 (jti1), writing the new plasma
// j_theta at the integer column i
template <typename T, int IO = IO_GLOBAL>
__device__ __forceinline__ cx<T> em_jt_avg(const Ctx<T>& c, const SetP<T>& s, const EmWin<T>& W, const EmB<T>& B,
                                           int row, int slot, bool write, cx<T> jti, cx<T> jti1,
                                           cx<T>* ring = nullptr) {
    cx<T> ja = jti + c.wp2h * (T(0.5) * (W.tpa[slot] + W.tma[slot]));
    cx<T> jb = jti1 + c.wp2h * (T(0.5) * (B.tpb[slot] + B.tmb[slot]));
    if (!c.g.open_r && row == c.g.nr) ja = jb = zero<T>();
    if constexpr (IO == IO_RING) {
        if (write) rput(c, ring, RG_JT, row, ja);
    } else {
        if (write && c.owner && c.o.col(c.i) >= 0) sto(s.ojt, eoff<T>(c.g, c.m, row, c.o.col(c.i)), ja);
    }
    if (c.x.i1 < 0) jb = zero<T>();
    return T(0.5) * (ja + jb);
}

// one march step of the electromagnetic set: outputs E_x(J=j+1), B_x(K=j)
// (and the exterior ghost at j = nr-1), T_r(K=j), T_theta(J=j)
template <typename T, int IO = IO_GLOBAL>
__device__ __forceinline__ void em_step(const Ctx<T>& c, const SetP<T>& s, EmWin<T>& W, const EmB<T>& B, int j,
                                        int r0, int r1, const RowInv<T>& ri, const EmRowX<T>& X,
                                        cx<T>* ring = nullptr) {
    constexpr bool RING = IO == IO_RING || IO == IO_RING_G;   // results to the ring
    constexpr bool GLOB = IO != IO_RING;                        // field values to the output planes
    constexpr int IOJ = IO == IO_RING_G ? IO_RING : IO;         // where the currents go
    const Geo& g = c.g;
    const int m = c.m;
    const T h = c.h;
    const int ocI = c.o.col(c.i);     // output column of integer column i
    const bool wI = c.owner && ocI >= 0;
    // rows stored to the output planes
    const int gr0 = IO == IO_RING_G ? c.gr0 : r0;
    const int gr1 = IO == IO_RING_G ? c.gr1 : r1;
    // ---- E_x^{n+1/2} at J = j+1
    if (j + 1 <= g.nr) {
        W.jx_n1 = em_jx<T, IOJ>(c, s, j + 1, W.ex0[1], j + 1 >= r0 && j + 1 < r1, W.pjx, W.pjxa, ring);
        W.ex1[2] = em_ex_new(c, W, B, j + 1, W.jx_n1, ri.irJ1);
        if constexpr (RING) {
            if (j + 1 >= r0 && j + 1 < r1) rput(c, ring, RG_EX, j + 1, W.ex1[2]);
        }
        if constexpr (GLOB) {
            if (j + 1 >= gr0 && j + 1 < gr1 && wI) sto(s.oex, eoff<T>(g, m, j + 1, ocI), W.ex1[2]);
        }
        if (j + 1 == g.nr) W.jx_nr = W.jx_n1;
    }
    if (j < 0) return;
    const bool own_row = j >= r0 && j < r1;
    const bool g_own = j >= gr0 && j < gr1;
    // ---- B_x^{n+1/2} at K = j
    if (j < g.nr) {
        W.bx1[1] = em_bx_new(c, W, B, ri.irK);
        if constexpr (RING) {
            if (own_row) rput(c, ring, RG_BX, j, W.bx1[1]);
        }
        if constexpr (GLOB) {
            if (g_own && wI) sto(s.obx, eoff<T>(g, m, j, ocI), W.bx1[1]);
        }
    }
    // ---- exterior ghost B_x^{n+1/2} at r_{nr+1/2} (Eq. em_r_open_bx)
    if (j == g.nr - 1) {
        cx<T> gh = zero<T>();
        if (g.open_r && c.live) {
            const int N = g.nr;
            const T kap = c.kap, cR = c.cR;
            cx<T> br_a = T(0.5) * (W.tpa[1] - W.tma[1]), br_b = T(0.5) * (B.tpb[1] - B.tmb[1]);
            cx<T> rx = c.inv_2h * (br_b - br_a);
            cx<T> ea = T(0.25) * ((W.tpa[1] + W.tma[1]) + (B.tpb[1] + B.tmb[1]));
            cx<T> ra = T(0.25) * ((W.rpa[0] + W.rma[0]) + (B.rpb[0] + B.rmb[0]));
            rx = rx - (T(0.5) * ri.irJ1) * (ea + imul(T(m), ra));
            cx<T> jt = zero<T>();
            if (c.plasma) {
                cx<T> jti, jti1;
                if constexpr (IO == IO_FROM_RING) {
                    // the first step's j_theta at row nr, columns i and i+1
                    jti = *rg(ring, RG_JT, N, c.lane);
                    jti1 = c.x.i1 >= 0 ? *rg(ring, RG_JT, N, min(c.lane + 1, WAVE - 1)) : zero<T>();
                } else {
                    jti = c.x.L(s.jt, m, N);
                    jti1 = c.x.R(s.jt, m, N);
                }
                jt = em_jt_avg(c, s, W, B, N, 1, false, jti, jti1);
            }
            if (s.jta) jt = jt + c.x.L(s.jta, m, N);
            rx = rx - T(0.5) * jt;
            gh = W.bx0[0] + kap * (W.bx0[1] - W.bx1[1]) + cR * rx;
        }
        W.bx1g = gh;
        if constexpr (RING) {
            if (r1 == g.nr + 1) rput(c, ring, RG_BX, g.nr, gh);
        }
        if constexpr (GLOB) {
            if (gr1 == g.nr + 1 && wI) sto(s.obx, eoff<T>(g, m, g.nr, ocI), gh);
        }
    }
    // ---- T_r transport on K = j
    if (j < g.nr) {
        cx<T> sp = zero<T>(), sm = zero<T>();
        cx<T> jra = zero<T>();
        const cx<T> jr1 = c.plasma ? c.x.Rn(X.jr) : zero<T>();   // uniform control flow here
        if (c.plasma) {
            jra = X.jr + c.wp2h * (T(0.5) * (W.rpa[0] + W.rma[0]));
            if constexpr (RING) {
                if (own_row) rput(c, ring, RG_JR, j, jra);
            } else {
                if (own_row && wI) sto(s.ojr, eoff<T>(g, m, j, ocI), jra);
            }
        }
        if (c.live) {
            cx<T> jr = zero<T>();
            if (c.plasma) {
                cx<T> jrb = jr1 + c.wp2h * (T(0.5) * (B.rpb[0] + B.rmb[0]));
                if (c.x.i1 < 0) jrb = zero<T>();
                jr = T(0.5) * (jra + jrb);
            }
            if (s.jra) jr = jr + X.jra;
            cx<T> gr = -imul(T(m) * ri.irK, W.bx1[1]) - jr;
            cx<T> pr = c.inv_dr * (W.ex1[2] - W.ex1[1]);
            sp = h * (gr + pr);
            sm = h * (gr - pr);
        }
        W.n_rpb = (c.x.i1 >= 0) ? W.rpa[0] + sp : zero<T>();       // T_r^+ at column i+1
        W.n_rma = B.rmb[0] + sm;                                     // T_r^- at column i
        cx<T> from_left = shfl_up1(W.n_rpb);
        cx<T> from_right = shfl_dn1(W.n_rma);
        W.n_rpa = (c.i == 0 && !g.per) ? zero<T>() : from_left;
        W.n_rmb = (c.x.i1 >= 0) ? from_right : zero<T>();
        if constexpr (RING) {
            // the lane's own column: T_r^+ came from the left neighbour
            if (own_row) {
                rput(c, ring, RG_TRP, j, W.n_rpa);
                rput(c, ring, RG_TRM, j, W.n_rma);
            }
        }
        if (GLOB && g_own) {
            if (c.owner && c.x.ir >= 0 && c.o.col(c.x.ir) >= 0) sto(s.otrp, eoff<T>(g, m, j, c.o.col(c.x.ir)), W.n_rpb);
            if (wI) sto(s.otrm, eoff<T>(g, m, j, ocI), W.n_rma);
            if (c.owner && c.i == 0 && !g.per && c.o.col(0) >= 0) sto(s.otrp, eoff<T>(g, m, j, c.o.col(0)), zero<T>());
        }
    }
    // ---- T_theta transport on J = j (exterior ghost B_x used at j = nr)
    {
        const bool zrow = (!g.open_r && j == g.nr) || (j == 0 && m != 1);
        cx<T> jt = zero<T>();
        const cx<T> jt1 = c.plasma ? c.x.Rn(X.jt) : zero<T>();   // uniform control flow here
        if (c.plasma) jt = em_jt_avg<T, IOJ>(c, s, W, B, j, 0, own_row, X.jt, jt1, ring);
        if (s.jta && c.live) jt = jt + X.jta;
        cx<T> sp = zero<T>(), sm = zero<T>();
        if (c.live && !zrow) {
            cx<T> gt, pt;
            if (j == 0) {
                gt = -(T(2) * c.inv_dr) * W.bx1[1] - jt;
                pt = imul(c.inv_dr, W.ex1[2]);
            } else {
                cx<T> bhi = (j == g.nr) ? W.bx1g : W.bx1[1];
                gt = -c.inv_dr * (bhi - W.bx1[0]) - jt;
                pt = imul(T(m) * ri.irJ, W.ex1[1]);
            }
            sp = h * (gt + pt);
            sm = h * (gt - pt);
        }
        if (zrow) {
            W.n_tpa = zero<T>();
            W.n_tmb = zero<T>();
        } else {
            W.n_tpa = B.tpb[0] + sp;                                      // T_theta^+ at column i
            W.n_tmb = (c.x.i1 >= 0) ? W.tma[0] + sm : zero<T>();          // T_theta^- at column i+1
        }
        cx<T> from_right = shfl_dn1(W.n_tpa);
        cx<T> from_left = shfl_up1(W.n_tmb);
        W.n_tpb = (c.x.i1 >= 0) ? from_right : zero<T>();
        W.n_tma = (c.i == 0 && !g.per) ? zero<T>() : from_left;
        if constexpr (RING) {
            if (own_row) {
                rput(c, ring, RG_TTP, j, W.n_tpa);
                rput(c, ring, RG_TTM, j, W.n_tma);
            }
        }
        if (GLOB && g_own) {
            if (wI) sto(s.ottp, eoff<T>(g, m, j, ocI), W.n_tpa);
            if (c.owner && c.x.ir >= 0 && c.o.col(c.x.ir) >= 0) sto(s.ottm, eoff<T>(g, m, j, c.o.col(c.x.ir)), W.n_tmb);
            if (c.owner && c.i == 0 && !g.per && c.o.col(0) >= 0) sto(s.ottm, eoff<T>(g, m, j, c.o.col(0)), zero<T>());
        }
    }
}

// exterior ghost B_theta at r_{nr+1/2} (Eq. em_r_open_bt), at j = nr - 1 after em_step
template <typename T, int IO = IO_GLOBAL>
__device__ __forceinline__ void em_ghost_bth(const Ctx<T>& c, const SetP<T>& s, const EmWin<T>& W, const EmB<T>& B,
                                             int r1, cx<T>* ring = nullptr) {
    const Geo& g = c.g;
    const int m = c.m, N = g.nr;
    const T dr = c.dr;
    cx<T> er_a = T(0.5) * (W.rpa[0] + W.rma[0]);
    cx<T> er_b = T(0.5) * (B.rpb[0] + B.rmb[0]);
    cx<T> er_l = shfl_up1(er_a);                        // E_r at column i-1
    cx<T> jx_l = shfl_up1(W.jx_nr);                     // j_x at (x_{i-1/2}, r_nr)
    if (c.i == 0 && !g.per) er_l = jx_l = zero<T>();
    cx<T> out = zero<T>();
    if (g.open_r) {
        const T rN = T(N) * dr;
        const T kap = c.kap, cR = c.cR;
        cx<T> I0 = T(0.5) * (W.rpa[0] - W.rma[0]);
        cx<T> I1 = T(0.5) * (W.n_rpa - W.n_rma);
        cx<T> G0 = T(0.5) * (W.rpa[1] - W.rma[1]);          // stored ghost (see em_load_next)
        cx<T> br = T(0.5) * (W.tpa[1] - W.tma[1]);          // B_r at (x_i, r_nr)
        cx<T> dxer = c.inv_2h * (er_b - er_l);
        cx<T> jxi = T(0.5) * (W.jx_nr + jx_l);
        cx<T> rt = -T(0.5) * dxer - (T(1) / (T(2) * rN)) * (T(0.5) * (I0 + G0) + imul(T(m), br)) + T(0.5) * jxi;
        out = I0 + kap * (G0 - I1) + cR * rt;
    }
    if constexpr (IO == IO_RING || IO == IO_RING_G) {
        // the second step reads the ghost row through T_r^+ alone
        if (r1 == g.nr + 1) rput(c, ring, RG_TRP, N, out);
    }
    if constexpr (IO != IO_RING) {
        const int oc = c.o.col(c.i);
        const int gr1 = IO == IO_RING_G ? c.gr1 : r1;
        if (c.owner && oc >= 0 && gr1 == g.nr + 1) {
            sto(s.otrp, eoff<T>(g, m, N, oc), out);
            sto(s.otrm, eoff<T>(g, m, N, oc), zero<T>());
        }
    }
}

template <typename T>
__device__ __forceinline__ void em_rotate(EmWin<T>& W) {
    W.rpa[0] = W.rpa[1]; W.rma[0] = W.rma[1];
    W.tpa[0] = W.tpa[1]; W.tma[0] = W.tma[1];
    W.ex0[0] = W.ex0[1];
    W.ex1[0] = W.ex1[1]; W.ex1[1] = W.ex1[2];
    W.bx0[0] = W.bx0[1];
    W.bx1[0] = W.bx1[1];
}

// Per-lane context of a marching wave of mode m over one strip: column of
// the lane (halo lanes wrap with periodic x; otherwise they are clamped, and
// their results only reach owned lanes through terms the x boundary zeroes),
// ownership and the step's constants.  A strip owns OWNC columns after LH
// left-halo lanes (the one-step marches: 61 after 1; the two-step march,
// whose second step needs the first step's results one lane further out on
// each side: 58 after 2).  xshift moves the strip's columns left (the second
// step of the two-step march with the moving window works in the frame the
// first step's shift made).
template <typename T, int OWNC = OWN, int LH = 1>
__device__ __forceinline__ Ctx<T> make_ctx(const FusedArgs<T>& a, int strip, int m, int lane, int xshift = 0) {
    const Geo& g = a.g;
    Ctx<T> c;
    c.g = g;
    c.m = m;
    c.lane = lane;
    c.rzero = false;
    c.gr0 = c.gr1 = 0;
    const int raw = strip * OWNC - LH - xshift + lane;
    const bool inrange = raw >= 0 && raw < g.nx;
    c.i = g.per ? ((raw % g.nx) + g.nx) % g.nx : (raw < 0 ? 0 : (raw >= g.nx ? g.nx - 1 : raw));
    c.owner = inrange && lane >= LH && lane < LH + OWNC;
    c.live = g.per || c.i < g.nx - 1;
    c.x.nr1 = g.nr + 1;
    c.x.ld = g.ld;
    c.x.i = c.i;
    c.x.i1 = (c.i + 1 < g.nx) ? c.i + 1 : (g.per ? 0 : -1);
    c.x.ir = c.x.i1;
    c.o.shift = a.window;
    c.o.nx = g.nx;
    c.h = T(g.h);
    c.dr = T(g.dr);
    c.inv_dr = T(1) / c.dr;
    c.inv_2dr = T(0.5) * c.inv_dr;
    c.kap = (c.dr - c.h) / (c.dr + c.h);
    c.cR = T(2) * c.h * c.dr / (c.dr + c.h);
    c.inv_2h = T(0.5) / c.h;
    c.wp2h = T(a.wp2 * g.h);
    c.plasma = a.plasma;
    return c;
}

// LDS exchange slots per lane: the 6 factors of the axion source (two such
// buffers, alternating by row)
constexpr int NS = 6;

// The factors of the axion source at K = j (Eqs. source_mode_zero,
// source_mode_m) of mode m from the window after em_step on row j: E_x and
// B_x at t^n, and the transport-variable form of the transverse part,
//   C{E_r, B_r} + C{E_th, B_th}
//     = 1/2 C{T_r^+ + b_th, T_th^+ + b_r} - 1/2 C{T_r^- - b_th, T_th^- - b_r}
// (exact; no cancellation between two large products for co-propagating
// waves); ex1_j is E_x^{n+1/2}(J = j), taken before em_step moved it on.
// The source is sum C_m{f0, f1} + C_m{f2, f3} + C_m{f4, f5}.
template <typename T>
__device__ __forceinline__ void sa_factors(const FusedArgs<T>& a, int m, const EmWin<T>& W, const EmB<T>& B,
                                           cx<T> ex1_j, cx<T>* f) {
    cx<T> bx_n = T(0.5) * (W.bx0[0] + W.bx1[1]);
    cx<T> exn0 = T(0.5) * (W.ex0[0] + ex1_j);
    cx<T> exn1 = T(0.5) * (W.ex0[1] + W.ex1[2]);
    cx<T> fEx = T(0.5) * (exn0 + exn1);
    cx<T> fBx = bx_n;
    cx<T> fPp = T(0.25) * (W.rpa[0] + B.rpb[0]);
    cx<T> fPm = T(-0.25) * (W.rma[0] + B.rmb[0]);
    cx<T> fQp = T(0.25) * ((W.tpa[0] + W.tpa[1]) + (B.tpb[0] + B.tpb[1]));
    cx<T> fQm = T(0.25) * ((W.tma[0] + W.tma[1]) + (B.tmb[0] + B.tmb[1]));
    if (m == 0) fBx = fBx + a.bx0;
    if (m == 1) {
        fPp = fPp + T(0.5) * a.bt1;
        fPm = fPm + T(0.5) * a.bt1;
        fQp = fQp + a.br1;
        fQm = fQm - a.br1;
    }
    f[0] = fEx; f[1] = fBx; f[2] = fPp; f[3] = fQp; f[4] = fPm; f[5] = fQm;
}

// ---------------------------------------------------------------------------
// kernel A: background set + axion
// ---------------------------------------------------------------------------
// AXT: kernel A advances the axion (T_a, phi); otherwise it writes S_a to a.sa
// for the marched axion current, which advances the axion instead.
template <typename T, int M, bool AXT>
__device__ __forceinline__ void fused_a_body(const FusedArgs<T>& a, int strip, int chunk, int rows) {
    const Geo g = a.g;
    const int wave = threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    const int r0 = chunk * rows;
    const int r1 = min(g.nr + 1, r0 + rows);
    const Ctx<T> c = make_ctx<T>(a, strip, wave, lane);

    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    // two exchange buffers [NS][M][WAVE], alternating by row: the one barrier
    // per row (after the writes) then also keeps the next row's writes behind
    // every wave's reads of this row
    cx<T>* const smS2 = reinterpret_cast<cx<T>*>(smem_raw);
    auto put = [&](cx<T>* base, int f, cx<T> v) { base[(f * M + wave) * WAVE + lane] = v; };
    auto get = [&](const cx<T>* base, int f, int k) { return base[(f * M + k) * WAVE + lane]; };

    const SetP<T>& s = a.s0;
    EmWin<T> W;
    cx<T> phw[3];     // phi^n at K = j-1, j, j+1
    const int m = wave;
    const T h = c.h;
    const T kap = c.kap;
    const int ocI = c.o.col(c.i);
    const bool wI = c.owner && ocI >= 0;
    // one halo row gives E_x(J = r0) and B_x(K = r0 - 1); the chunk holding the
    // exterior ghost row also needs E_x(J = nr - 1) for the ghost B_theta
    const int jstart = max(r0 - (r1 == g.nr + 1 ? 2 : 1), -1);
    // prime slot 1 with row jstart (so that the first em_load_next fills j+1)
    for (int q = 0; q < 2; ++q) {
        W.rpa[q] = W.rma[q] = zero<T>();
        W.tpa[q] = W.tma[q] = zero<T>();
        W.ex0[q] = W.bx0[q] = W.bx1[q] = zero<T>();
    }
    W.ex1[0] = W.ex1[1] = W.ex1[2] = zero<T>();
    W.bx1g = W.jx_n1 = W.jx_nr = zero<T>();
    phw[0] = phw[1] = phw[2] = zero<T>();
    // phi on half row k (the exterior ghost on row nr with the open boundary)
    auto phi_row = [&](int k) {
        if (k < g.nr) return c.x.L(a.phi, m, k);
        if (k == g.nr && g.open_r) return c.x.L(a.phi, m, g.nr);
        return zero<T>();
    };
    constexpr bool axt = AXT;
    if (jstart >= 0) {
        em_take(c, W, em_fetch(c, s, jstart), jstart, g.nr);   // row jstart into slot 1
        if (axt) {
            phw[2] = (jstart < g.nr) ? c.x.L(a.phi, m, jstart) : zero<T>();
            if (jstart - 1 >= 0) phw[1] = c.x.L(a.phi, m, jstart - 1);
        }
    }
    // FP64 issues the axion transport loads of row j with the row's other
    // loads; FP32 loads them where they are used, to keep four waves per SIMD
    constexpr bool HOIST = sizeof(T) == 8;
    // rows [r0, r1) are owned; the last iteration is r1 - 1 except for the
    // chunk holding the exterior ghost row, which ends on row nr
    const int jend = r1 == g.nr + 1 ? g.nr : r1 - 1;
    for (int j = jstart; j <= jend; ++j) {
        // ---------------- shift the window and load row j+1
        em_rotate(W);
        phw[0] = phw[1]; phw[1] = phw[2];
        if (axt) phw[2] = phi_row(j + 1);
        em_take(c, W, em_fetch(c, s, j + 1), j + 1, g.nr);
        const EmRowX<T> X = em_fetch_x(c, s, j);
        cx<T> tap_a = zero<T>(), tam_a = zero<T>();
        if (HOIST && axt && j >= 0 && j < g.nr) {
            tap_a = c.x.L(a.tap, m, j);
            tam_a = c.x.L(a.tam, m, j);
        }
        const EmB<T> B = em_bvals(c, W);
        const cx<T> ex1_j = W.ex1[1];
        const RowInv<T> ri = row_inv(c, j);
        em_step(c, s, W, B, j, r0, r1, ri, X);
        if (j < 0) continue;
        const bool own_row = j >= r0 && j < r1;
        if (j == g.nr - 1) em_ghost_bth(c, s, W, B, r1);

        // ---------------- axion source S_a at K = j (Eqs. source_mode_zero/_m)
        cx<T>* const smS = smS2 + (j & 1) * (NS * M * WAVE);
        cx<T> Sa = zero<T>();
        cx<T> ga = zero<T>();
        if (j < g.nr) {
            cx<T> f[NS];
            sa_factors(a, m, W, B, ex1_j, f);
#pragma unroll
            for (int q = 0; q < NS; ++q) put(smS, q, f[q]);
        }
        __syncthreads();
        if (j < g.nr) {
            auto gS = [&](int f, int k) { return get(smS, f, k); };
            conv_pair<T, M>(gS, 0, 1, m, Sa, T(1));
            conv_pair<T, M>(gS, 2, 3, m, Sa, T(1));
            conv_pair<T, M>(gS, 4, 5, m, Sa, T(1));
            if (!c.live) Sa = zero<T>();
            if (!axt) {
                if (own_row && c.owner) sto(a.sa, eoff<T>(g, m, j, c.i), Sa);
                continue;
            }
            // ---------------- Gamma_a, T_a transport, phi (Eqs. Ta_plus/minus_update, phi_update)
            cx<T> p = phw[1];
            cx<T> up = phw[2];
            cx<T> dn = (j > 0) ? phw[0] : zero<T>();
            if (c.live)
                ga = (c.inv_dr * c.inv_dr) * (up - T(2) * p + dn) + (c.inv_2dr * ri.irK) * (up - dn)
                     - (T(m * m) * ri.irK * ri.irK + T(a.ma2)) * p + T(a.s_phi) * Sa;
            if (!HOIST) {
                tap_a = c.x.L(a.tap, m, j);
                tam_a = c.x.L(a.tam, m, j);
            }
            const cx<T> tam_b = c.x.Rn(tam_a);   // uniform control flow here
            cx<T> nap_b = (c.x.i1 >= 0) ? tap_a + h * ga : zero<T>();     // T_a^+ at column i+1
            cx<T> nam_a = tam_b + h * ga;                                  // T_a^- at column i
            cx<T> l = shfl_up1(nap_b), r = shfl_dn1(nam_a);
            cx<T> nap_a = (c.i == 0 && !g.per) ? zero<T>() : l;
            cx<T> nam_b = (c.x.i1 >= 0) ? r : zero<T>();
            cx<T> p1 = zero<T>();
            if (c.live) p1 = p + (h / T(4)) * (nap_a + nap_b + nam_a + nam_b);
            if (own_row) {
                if (c.owner && c.x.ir >= 0 && c.o.col(c.x.ir) >= 0) sto(a.otap, eoff<T>(g, m, j, c.o.col(c.x.ir)), nap_b);
                if (wI) {
                    sto(a.otam, eoff<T>(g, m, j, ocI), nam_a);
                    sto(a.ophi, eoff<T>(g, m, j, ocI), p1);
                }
                if (c.owner && c.i == 0 && !g.per && c.o.col(0) >= 0) sto(a.otap, eoff<T>(g, m, j, c.o.col(0)), zero<T>());
            }
            if (j == g.nr - 1 && wI && r1 == g.nr + 1) {
                // exterior ghost phi at r_{nr+1/2}: outgoing-wave condition, two-level centring
                cx<T> G = phw[2];
                cx<T> Gn = G;
                if (g.open_r) Gn = c.live ? (p + kap * (G - p1)) : zero<T>();
                sto(a.ophi, eoff<T>(g, m, g.nr, ocI), Gn);
            }
        }
    }
    // moving window: the owner of the last cell zero-fills the last column
    if (a.window && c.owner && c.i == g.nx - 1) {
        for (int row = r0; row < r1; ++row) {
            const uint32_t e = eoff<T>(g, m, row, g.nx - 1);
            sto(s.otrp, e, zero<T>()); sto(s.otrm, e, zero<T>()); sto(s.ottp, e, zero<T>()); sto(s.ottm, e, zero<T>());
            sto(s.oex, e, zero<T>()); sto(s.obx, e, zero<T>());
            if (c.plasma) { sto(s.ojx, e, zero<T>()); sto(s.ojr, e, zero<T>()); sto(s.ojt, e, zero<T>()); }
            sto(a.ophi, e, zero<T>()); sto(a.otap, e, zero<T>()); sto(a.otam, e, zero<T>());
        }
    }
}

// ---------------------------------------------------------------------------
// kernel AX: the background set, the axion source, the axion advance and the
// axion current in one r-march (the regenerated set follows in kernel B)
// ---------------------------------------------------------------------------
// A workgroup is M wavefronts (one per mode) over one strip and a chunk of
// rows, as kernel A.  On row j a wave advances the background set (em_step),
// forms S_a at K = j through the LDS exchange of its factors, advances the
// axion on K = j (Gamma_a, the T_a^+- transport and phi^{n+1}), and then
// builds the per-point combinations of K = j and J = j that the axion current
// reads from the values already in its registers: the old and new transport
// variables, E_x and B_x at both levels, and the old and new axion.  Nothing
// of the background set is read twice and S_a never leaves the chip.  The
// current's factors of j_a,x and j_a,theta at row j and of j_a,r at K = j - 1
// (which needs T_theta^{n+1} on J = j) go through a second LDS exchange.  A
// chunk [r0, r1) owns the rows of the background set, the axion and j_a,x,
// j_a,theta in [r0, r1), and the j_a,r rows K in [r0 - 1, r1 - 1) (so no row
// above the chunk is needed); it marches from the halo row r0 - 2, whose
// E_x^{n+1/2}(J = r0 - 1) completes S_a and the row windows of K = r0 - 1.
// LDS: area X holds the 6 factors of S_a, area Y the 18 of j_a; two barriers
// per row order the writes of one row after every wave's reads of the last.
constexpr int NJ = 18;

// Output stores of the axion and its current: streaming in FP64 (kernel B,
// which runs next, measured faster with T_a, phi and j_a kept out of the
// caches), plain in FP32.
template <typename T>
__device__ __forceinline__ void sto_ax(cx<T>* p, uint32_t o, cx<T> v) {
    cx<T>* q = (cx<T>*)((g_char*)(p) + o);
    if constexpr (sizeof(T) == 8) st_nt(q, v);
    else st(q, v);
}

template <typename T, int M>
__device__ __forceinline__ void fused_ax_body(const FusedArgs<T>& a, int strip, int chunk, int rows) {
    const Geo g = a.g;
    const int wave = threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    const int r0 = chunk * rows;
    const int r1 = min(g.nr + 1, r0 + rows);
    const Ctx<T> c = make_ctx<T>(a, strip, wave, lane);
    const int m = wave;

    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* const smX = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* const smY = smX + NS * M * WAVE;
    auto put = [&](cx<T>* base, int f, cx<T> v) { base[(f * M + wave) * WAVE + lane] = v; };
    auto get = [&](const cx<T>* base, int f, int k) { return base[(f * M + k) * WAVE + lane]; };
    // out += C{f0, f1} - C{f2, f3} + C{f4, f5} over the six factors from slot f0
    auto conv3 = [&](int f0, cx<T>& out) {
        cx<T> A[M], B[M];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
#pragma unroll
            for (int k = 0; k < M; ++k) { A[k] = get(smY, f0 + 2 * q, k); B[k] = get(smY, f0 + 2 * q + 1, k); }
            conv_one<T, M>(A, B, m, out, q == 1 ? T(-1) : T(1));
        }
    };

    const SetP<T>& s = a.s0;
    EmWin<T> W;
    for (int q = 0; q < 2; ++q) {
        W.rpa[q] = W.rma[q] = zero<T>();
        W.tpa[q] = W.tma[q] = zero<T>();
        W.ex0[q] = W.bx0[q] = W.bx1[q] = zero<T>();
    }
    W.ex1[0] = W.ex1[1] = W.ex1[2] = zero<T>();
    W.bx1g = W.jx_n1 = W.jx_nr = zero<T>();
    W.pjx = W.pjxa = zero<T>();
    cx<T> phw[3];     // phi^n at K = j-1, j, j+1
    phw[0] = phw[1] = phw[2] = zero<T>();
    const T h = c.h;
    const T kap = c.kap;
    const T sj = T(a.s_j);
    const bool has1 = c.x.i1 >= 0;
    const cur::FacC<T> fc{m, parity<T>(m), tghost<T>(m), c.dr, c.inv_dr, a.bx0, a.br1, a.bt1};
    auto phi_row = [&](int k) {
        if (k < 0) return zero<T>();
        if (k < g.nr) return c.x.L(a.phi, m, k);
        if (k == g.nr && g.open_r) return c.x.L(a.phi, m, g.nr);
        return zero<T>();
    };
    const int jstart = max(r0 - 2, -1);
    // first row whose S_a, axion advance and row windows are complete
    const int jfull = max(r0 - 1, 0);
    if (jstart >= 0) {
        em_take(c, W, em_fetch(c, s, jstart), jstart, g.nr);   // row jstart into slot 1
        phw[2] = phi_row(jstart);
        phw[1] = phi_row(jstart - 1);
    }
    cur::KRow<T> kp = cur::zero_k<T>();   // K row j - 1
    cur::JRow<T> jp = cur::zero_j<T>();   // J row j - 1
    const int jend = r1 == g.nr + 1 ? g.nr : r1 - 1;
    for (int j = jstart; j <= jend; ++j) {
        // ---------------- shift the window and load row j+1 (issued together
        // with the row's currents and T_a, and consumed at once: a prefetch of
        // the next row one iteration ahead, kept across the axion part,
        // measured slower, its registers costing a wave per SIMD in FP32 and
        // spills in FP64)
        em_rotate(W);
        phw[0] = phw[1]; phw[1] = phw[2];
        phw[2] = phi_row(j + 1);
        em_take(c, W, em_fetch(c, s, j + 1), j + 1, g.nr);
        // FP64 issues the T_a loads of row j with the row's other loads; FP32
        // loads them where they are used (as kernel A)
        constexpr bool HOIST = sizeof(T) == 8;
        cx<T> tap_a = zero<T>(), tam_a = zero<T>();
        if (HOIST && j >= jfull && j < g.nr) {
            tap_a = c.x.L(a.tap, m, j);
            tam_a = c.x.L(a.tam, m, j);
        }
        const EmRowX<T> X = em_fetch_x(c, s, j);
        const EmB<T> B = em_bvals(c, W);
        const cx<T> ex1_j = W.ex1[1];
        const RowInv<T> ri = row_inv(c, j);
        em_step(c, s, W, B, j, r0, r1, ri, X);
        if (j < 0) continue;
        if (j == g.nr - 1) em_ghost_bth(c, s, W, B, r1);
        if (j < jfull) continue;      // the same for every wave of the workgroup
        const bool own_row = j >= r0 && j < r1;

        // ---------------- axion source S_a at K = j (Eqs. source_mode_zero/_m)
        if (j < g.nr) {
            cx<T> bx_n = T(0.5) * (W.bx0[0] + W.bx1[1]);
            cx<T> exn0 = T(0.5) * (W.ex0[0] + ex1_j);
            cx<T> exn1 = T(0.5) * (W.ex0[1] + W.ex1[2]);
            cx<T> fEx = T(0.5) * (exn0 + exn1);
            cx<T> fBx = bx_n;
            cx<T> fPp = T(0.25) * (W.rpa[0] + B.rpb[0]);
            cx<T> fPm = T(-0.25) * (W.rma[0] + B.rmb[0]);
            cx<T> fQp = T(0.25) * ((W.tpa[0] + W.tpa[1]) + (B.tpb[0] + B.tpb[1]));
            cx<T> fQm = T(0.25) * ((W.tma[0] + W.tma[1]) + (B.tmb[0] + B.tmb[1]));
            if (m == 0) fBx = fBx + a.bx0;
            if (m == 1) {
                fPp = fPp + T(0.5) * a.bt1;
                fPm = fPm + T(0.5) * a.bt1;
                fQp = fQp + a.br1;
                fQm = fQm - a.br1;
            }
            put(smX, 0, fEx); put(smX, 1, fBx); put(smX, 2, fPp); put(smX, 3, fQp); put(smX, 4, fPm); put(smX, 5, fQm);
        }
        __syncthreads();
        cur::KRow<T> kc = cur::zero_k<T>();
        if (j < g.nr) {
            cx<T> Sa = zero<T>();
            cx<T> A[M], Bq[M];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
#pragma unroll
                for (int k = 0; k < M; ++k) { A[k] = get(smX, 2 * q, k); Bq[k] = get(smX, 2 * q + 1, k); }
                conv_one<T, M>(A, Bq, m, Sa, T(1));
            }
            if (!c.live) Sa = zero<T>();
            // ---------------- Gamma_a, T_a transport, phi (Eqs. Ta_plus/minus_update, phi_update)
            const cx<T> p = phw[1];
            const cx<T> up = phw[2];
            const cx<T> dn = (j > 0) ? phw[0] : zero<T>();
            cx<T> ga = zero<T>();
            if (c.live)
                ga = (c.inv_dr * c.inv_dr) * (up - T(2) * p + dn) + (c.inv_2dr * ri.irK) * (up - dn)
                     - (T(m * m) * ri.irK * ri.irK + T(a.ma2)) * p + T(a.s_phi) * Sa;
            if (!HOIST) {
                tap_a = c.x.L(a.tap, m, j);
                tam_a = c.x.L(a.tam, m, j);
            }
            const cx<T> tam_b = c.x.Rn(tam_a);   // uniform control flow here
            const cx<T> nap_b = has1 ? tap_a + h * ga : zero<T>();     // T_a^+ at column i+1
            const cx<T> nam_a = tam_b + h * ga;                         // T_a^- at column i
            const cx<T> l = shfl_up1(nap_b), rr = shfl_dn1(nam_a);
            const cx<T> nap_a = (c.i == 0 && !g.per) ? zero<T>() : l;
            const cx<T> nam_b = has1 ? rr : zero<T>();
            cx<T> p1 = zero<T>();
            if (c.live) p1 = p + (h / T(4)) * (nap_a + nap_b + nam_a + nam_b);
            // (with the moving window every new value lands one column left)
            const int oc = c.o.col(c.i);
            if (own_row && c.owner) {
                if (has1 && c.o.col(c.x.i1) >= 0) sto_ax(a.otap, eoff<T>(g, m, j, c.o.col(c.x.i1)), nap_b);
                if (oc >= 0) {
                    sto_ax(a.otam, eoff<T>(g, m, j, oc), nam_a);
                    sto_ax(a.ophi, eoff<T>(g, m, j, oc), p1);
                    if (c.i == 0 && !g.per) sto_ax(a.otap, eoff<T>(g, m, j, oc), zero<T>());
                }
                if (j == g.nr - 1 && oc >= 0) {
                    // exterior ghost phi at r_{nr+1/2}: outgoing-wave condition, two-level centring
                    cx<T> Gn = up;
                    if (g.open_r) Gn = c.live ? (p + kap * (up - p1)) : zero<T>();
                    sto_ax(a.ophi, eoff<T>(g, m, g.nr, oc), Gn);
                }
            }
            // ---------------- the current's combinations on K = j
            const T q = T(0.5);
            kc.bxn = q * (W.bx0[0] + W.bx1[1]);
            kc.er0 = q * (W.rpa[0] + W.rma[0]);
            kc.P = q * (W.rpa[0] + W.n_rpa);
            kc.N = q * (W.rma[0] + W.n_rma);
            kc.ph0 = p;
            kc.up = nap_a;
            kc.wm = nam_a;
            kc.dt0 = q * (q * (tap_a + tam_a) + q * (nap_a + nam_a));
            kc.phm = q * (p + p1);
        }
        // ... and on J = j
        cur::JRow<T> jc;
        {
            const T q = T(0.5);
            jc.et0 = q * (W.tpa[0] + W.tma[0]);
            jc.Qp = q * (W.tpa[0] + W.n_tpa);
            jc.Qm = q * (W.tma[0] + W.n_tma);
            jc.ex = ex1_j;
        }
        // ---------------- axion current (Eqs. jax_mode, jat_mode at row j; jar_mode at K = j - 1)
        const bool do_xt = own_row;
        const bool do_r = j >= r0 && j >= 1;
        const bool calc_xt = do_xt && c.live && j < g.nr;
        const bool calc_r = do_r && c.live;
        {
            const cur::NbX<T> nx = cur::nb_x(kp, kc, jc, has1);
            if (calc_xt) {
                cx<T> f[6];
                cur::fac_x(fc, j, kp, kc, jc, nx, f);
#pragma unroll
                for (int k = 0; k < 6; ++k) put(smY, k, f[k]);
            }
        }
        {
            const cur::NbT<T> nt = cur::nb_t(kp, kc, jc, has1);
            if (calc_xt) {
                cx<T> f[6];
                cur::fac_t(fc, j, kp, kc, jc, nt, f);
#pragma unroll
                for (int k = 0; k < 6; ++k) put(smY, 6 + k, f[k]);
            }
        }
        {
            const cur::NbR<T> nr = cur::nb_r(kp, jp, jc, has1);
            if (calc_r) {
                cx<T> f[6];
                cur::fac_r(fc, j - 1, kp, jp, jc, nr, f);
#pragma unroll
                for (int k = 0; k < 6; ++k) put(smY, 12 + k, f[k]);
            }
        }
        __syncthreads();
        if (do_xt && c.owner) {
            cx<T> ox = zero<T>(), ot = zero<T>();
            if (calc_xt) {
                conv3(0, ox);
                conv3(6, ot);
            }
            sto_ax(a.jax, eoff<T>(g, m, j, c.i), sj * ox);
            sto_ax(a.jat, eoff<T>(g, m, j, c.i), sj * ot);
        }
        if (do_r && c.owner) {
            cx<T> orr = zero<T>();
            if (calc_r) conv3(12, orr);
            sto_ax(a.jar, eoff<T>(g, m, j - 1, c.i), sj * orr);
        }
        kp = kc;
        jp = jc;
    }
    // moving window: the owner of the last cell zero-fills the last column of
    // the new state (j_a stays at the old state's columns, where kernel B reads it)
    if (a.window && c.owner && c.i == g.nx - 1) {
        for (int row = r0; row < r1; ++row) {
            const uint32_t e = eoff<T>(g, m, row, g.nx - 1);
            sto(s.otrp, e, zero<T>()); sto(s.otrm, e, zero<T>()); sto(s.ottp, e, zero<T>()); sto(s.ottm, e, zero<T>());
            sto(s.oex, e, zero<T>()); sto(s.obx, e, zero<T>());
            if (c.plasma) { sto(s.ojx, e, zero<T>()); sto(s.ojr, e, zero<T>()); sto(s.ojt, e, zero<T>()); }
            sto(a.ophi, e, zero<T>()); sto(a.otap, e, zero<T>()); sto(a.otam, e, zero<T>());
        }
    }
}

// ---------------------------------------------------------------------------
// kernel B (and the electromagnetic-only step): one set, marched in r
// ---------------------------------------------------------------------------
template <typename T, int WHICH>
__device__ __forceinline__ void em_body(const FusedArgs<T>& a, int strip, int chunk, int m, int rows) {
    const Geo g = a.g;
    const int lane = threadIdx.x;
    const int r0 = chunk * rows;
    const int r1 = min(g.nr + 1, r0 + rows);
    const Ctx<T> c = make_ctx<T>(a, strip, m, lane);
    const SetP<T>& s = WHICH ? a.s1 : a.s0;
    EmWin<T> W;
    for (int q = 0; q < 2; ++q) {
        W.rpa[q] = W.rma[q] = zero<T>();
        W.tpa[q] = W.tma[q] = zero<T>();
        W.ex0[q] = W.bx0[q] = W.bx1[q] = zero<T>();
    }
    W.ex1[0] = W.ex1[1] = W.ex1[2] = zero<T>();
    W.bx1g = W.jx_n1 = W.jx_nr = zero<T>();
    // one halo row gives E_x(J = r0) and B_x(K = r0 - 1); the chunk holding the
    // exterior ghost row also needs E_x(J = nr - 1) for the ghost B_theta
    const int jstart = max(r0 - (r1 == g.nr + 1 ? 2 : 1), -1);
    W.pjx = W.pjxa = zero<T>();
    if (jstart >= 0) em_take(c, W, em_fetch(c, s, jstart), jstart, g.nr);
    EmPf<T> pf = em_fetch(c, s, jstart + 1);
    // rows [r0, r1) are owned; the last iteration is r1 - 1 except for the
    // chunk holding the exterior ghost row, which ends on row nr
    const int jend = r1 == g.nr + 1 ? g.nr : r1 - 1;
    for (int j = jstart; j <= jend; ++j) {
        em_rotate(W);
        em_take(c, W, pf, j + 1, g.nr);
        if (j < jend) pf = em_fetch(c, s, j + 2);   // next row's loads overlap this row's work
        const EmRowX<T> X = em_fetch_x(c, s, j);
        const EmB<T> B = em_bvals(c, W);
        em_step(c, s, W, B, j, r0, r1, row_inv(c, j), X);
        if (j == g.nr - 1) em_ghost_bth(c, s, W, B, r1);
    }
    if (a.window && c.owner && c.i == g.nx - 1) {
        for (int row = r0; row < r1; ++row) {
            const uint32_t e = eoff<T>(g, m, row, g.nx - 1);
            sto(s.otrp, e, zero<T>()); sto(s.otrm, e, zero<T>()); sto(s.ottp, e, zero<T>()); sto(s.ottm, e, zero<T>());
            sto(s.oex, e, zero<T>()); sto(s.obx, e, zero<T>());
            if (c.plasma) { sto(s.ojx, e, zero<T>()); sto(s.ojr, e, zero<T>()); sto(s.ojt, e, zero<T>()); }
        }
    }
}

// ---------------------------------------------------------------------------
// two steps of one set in one pass (temporal blocking): a workgroup of two
// waves over one (strip, chunk, mode).  Wave 0 marches the first step as the
// one-step march does, over the rows [p0, p1) that the second step reads, and
// puts its results in an LDS ring of 4 rows instead of the state planes; wave
// 1 marches the second step two rows behind, reading the first step's results
// from the ring (and the second step's extra current from its plane), and
// stores the rows [r0, r1) of its 58 owned columns.  One barrier per row: at
// tick t wave 0 writes rows t and t+1, wave 1 reads rows t-2 and t-1, and the
// barrier ends the tick, so every value wave 1 reads was written a tick before
// and no slot is rewritten while it is read.  The set's planes are read and
// written once per two steps; the arithmetic of each step is that of
// em_step, in the same order, so the result equals two one-step marches.
// ---------------------------------------------------------------------------
// PL = 0: the set carries no plasma currents (a.plasma is 0), which the
// compiler then drops (in FP32 126 VGPRs instead of 140: four waves per SIMD
// instead of three).
template <typename T, int WHICH, int PL>
__device__ __forceinline__ void em2_body(const FusedArgs<T>& a, int strip, int chunk, int m, int rows) {
    const Geo g = a.g;
    // 0: first step, 1: second step (wave-uniform, so each wave takes one
    // loop on a scalar branch and meets exactly that loop's barriers)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x % WAVE;
    const int r0 = chunk * rows;
    const int r1 = min(g.nr + 1, r0 + rows);
    // with the moving window the first step's result of lane k lands one
    // column to the left, so the second step's strip starts one column
    // further left and lane k still reads ring slot k; the first step's lanes
    // on column nx put the zero-filled column the window brings in
    Ctx<T> c = make_ctx<T, kPairOwn, 2>(a, strip, m, lane, wave == 1 ? a.window : 0);
    if (!PL) c.plasma = 0;
    if (wave == 0 && a.window) c.rzero = strip * kPairOwn - 2 + lane >= g.nx;
    const SetP<T>& s = WHICH ? a.s1 : a.s0;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* const ring = reinterpret_cast<cx<T>*>(smem_raw);
    // the second step's iterations, as in em_body
    const int jsc = max(r0 - (r1 == g.nr + 1 ? 2 : 1), -1);
    const int jec = r1 == g.nr + 1 ? g.nr : r1 - 1;
    // the first step owns the rows the second reads, [p0, p1)
    const int p0 = max(jsc, 0);
    const int p1 = min(jec + 2, g.nr + 1);
    const int jsp = max(p0 - (p1 == g.nr + 1 ? 2 : 1), -1);
    const int jep = p1 == g.nr + 1 ? g.nr : p1 - 1;
    EmWin<T> W;
    for (int q = 0; q < 2; ++q) {
        W.rpa[q] = W.rma[q] = zero<T>();
        W.tpa[q] = W.tma[q] = zero<T>();
        W.ex0[q] = W.bx0[q] = W.bx1[q] = zero<T>();
    }
    W.ex1[0] = W.ex1[1] = W.ex1[2] = zero<T>();
    W.bx1g = W.jx_n1 = W.jx_nr = zero<T>();
    W.pjx = W.pjxa = zero<T>();
    // both loops run the ticks jsp .. jec + 2, one barrier each
    if (wave == 0) {
        if (jsp >= 0) em_take(c, W, em_fetch(c, s, jsp), jsp, g.nr);
        EmPf<T> pf = em_fetch(c, s, jsp + 1);
        for (int t = jsp; t <= jec + 2; ++t) {
            if (t <= jep) {
                em_rotate(W);
                em_take(c, W, pf, t + 1, g.nr);
                if (t < jep) pf = em_fetch(c, s, t + 2);
                const EmRowX<T> X = em_fetch_x(c, s, t);
                const EmB<T> B = em_bvals(c, W);
                em_step<T, IO_RING>(c, s, W, B, t, p0, p1, row_inv(c, t), X, ring);
                if (t == g.nr - 1) em_ghost_bth<T, IO_RING>(c, s, W, B, p1, ring);
            }
            __syncthreads();
        }
    } else {
        // the second step's extra currents are those of the following step
        SetP<T> s2 = s;
        s2.jxa = s.jxb; s2.jra = s.jrb; s2.jta = s.jtb;
        // its loads from the current planes run one iteration ahead: j_x of
        // row j+1 and j_r, j_theta of row j are in flight since iteration j-1
        cx<T> xa_pre = em_xa(c, s2, jsc);
        cx<T> xa_nxt = em_xa(c, s2, jsc + 1);
        EmRowX<T> xrt = em_xrt(c, s2, jsc);
        for (int t = jsp; t <= jec + 2; ++t) {
            const int j = t - 2;
            if (j == jsc - 1) {
                if (jsc >= 0) em_take(c, W, em_fetch_ring(c, ring, jsc, xa_pre), jsc, g.nr);
            } else if (j >= jsc && j <= jec) {
                em_rotate(W);
                em_take(c, W, em_fetch_ring(c, ring, j + 1, xa_nxt), j + 1, g.nr);
                const EmRowX<T> X = em_fetch_x_ring(c, ring, j, xrt);
                if (j < jec) {
                    xa_nxt = em_xa(c, s2, j + 2);
                    xrt = em_xrt(c, s2, j + 1);
                }
                const EmB<T> B = em_bvals(c, W);
                em_step<T, IO_FROM_RING>(c, s2, W, B, j, r0, r1, row_inv(c, j), X, ring);
                if (j == g.nr - 1) em_ghost_bth<T, IO_FROM_RING>(c, s2, W, B, r1, ring);
            }
            __syncthreads();
        }
        // moving window: the owner of the last cell zero-fills the last column
        // of the new state, as the one-step march does
        if (a.window && c.owner && c.i == g.nx - 1) {
            for (int row = r0; row < r1; ++row) {
                const uint32_t e = eoff<T>(g, m, row, g.nx - 1);
                sto(s.otrp, e, zero<T>()); sto(s.otrm, e, zero<T>()); sto(s.ottp, e, zero<T>()); sto(s.ottm, e, zero<T>());
                sto(s.oex, e, zero<T>()); sto(s.obx, e, zero<T>());
                if (c.plasma) { sto(s.ojx, e, zero<T>()); sto(s.ojr, e, zero<T>()); sto(s.ojt, e, zero<T>()); }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// two steps of the background set with the axion source of each (temporal
// blocking of kernel A): a workgroup of 2M waves over one (strip, chunk).
// Waves 0..M-1 run the first step of modes 0..M-1 as kernel A does, putting
// their rows into a per-mode LDS ring and their field values (T^+-, E_x, B_x,
// which the axion kernel reads) into the intermediate planes; waves M..2M-1
// run the second step two rows behind from the ring, into the output planes.
// Each group forms S_a of its step through its own exchange area.  Two
// barriers per row: after the rows' ring writes and factors, and after the
// convolutions, so a factor slot is rewritten only once every wave of its
// group has read it; the ring keeps the lag and slot rules of em2_body.
// ---------------------------------------------------------------------------
template <typename T, int M>
__device__ __forceinline__ void fused_a2_body(const FusedArgs<T>& a, int strip, int chunk, int rows) {
    const Geo g = a.g;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int grp = wave / M;        // 0: first step, 1: second step (wave-uniform)
    const int m = wave - grp * M;
    const int lane = threadIdx.x % WAVE;
    const int r0 = chunk * rows;
    const int r1 = min(g.nr + 1, r0 + rows);
    Ctx<T> c = make_ctx<T, kPairOwn, 2>(a, strip, m, lane);
    c.gr0 = r0;
    c.gr1 = r1;
    const SetP<T>& s = a.s0;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* const base = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* const ring = base + m * (RG_N * RING_ROWS * WAVE);
    cx<T>* const xch = base + M * (RG_N * RING_ROWS * WAVE);   // [2 groups][NS][M][WAVE]
    auto put = [&](int f, cx<T> v) { xch[((grp * NS + f) * M + m) * WAVE + lane] = v; };
    auto gS = [&](int f, int k) { return xch[((grp * NS + f) * M + k) * WAVE + lane]; };
    // the rows of the two steps, as in em2_body
    const int jsc = max(r0 - (r1 == g.nr + 1 ? 2 : 1), -1);
    const int jec = r1 == g.nr + 1 ? g.nr : r1 - 1;
    const int p0 = max(jsc, 0);
    const int p1 = min(jec + 2, g.nr + 1);
    const int jsp = max(p0 - (p1 == g.nr + 1 ? 2 : 1), -1);
    const int jep = p1 == g.nr + 1 ? g.nr : p1 - 1;
    EmWin<T> W;
    for (int q = 0; q < 2; ++q) {
        W.rpa[q] = W.rma[q] = zero<T>();
        W.tpa[q] = W.tma[q] = zero<T>();
        W.ex0[q] = W.bx0[q] = W.bx1[q] = zero<T>();
    }
    W.ex1[0] = W.ex1[1] = W.ex1[2] = zero<T>();
    W.bx1g = W.jx_n1 = W.jx_nr = zero<T>();
    W.pjx = W.pjxa = zero<T>();
    // S_a of row k from the factors the group put: stored for the rows
    // [r0, r1) (unshifted columns, as kernel A)
    auto sa_store = [&](int k, cx<T>* out) {
        cx<T> Sa = zero<T>();
        conv_pair<T, M>(gS, 0, 1, m, Sa, T(1));
        conv_pair<T, M>(gS, 2, 3, m, Sa, T(1));
        conv_pair<T, M>(gS, 4, 5, m, Sa, T(1));
        if (!c.live) Sa = zero<T>();
        if (k >= r0 && k < r1 && c.owner) sto(out, eoff<T>(g, m, k, c.i), Sa);
    };
    if (grp == 0) {
        // the first step's field planes go to the intermediate planes
        SetP<T> sp = s;
        sp.otrp = a.mtrp; sp.otrm = a.mtrm; sp.ottp = a.mttp; sp.ottm = a.mttm; sp.oex = a.mex; sp.obx = a.mbx;
        if (jsp >= 0) em_take(c, W, em_fetch(c, s, jsp), jsp, g.nr);
        EmPf<T> pf = em_fetch(c, s, jsp + 1);
        for (int t = jsp; t <= jec + 2; ++t) {
            bool sa_row = false;
            if (t <= jep) {
                em_rotate(W);
                em_take(c, W, pf, t + 1, g.nr);
                if (t < jep) pf = em_fetch(c, s, t + 2);
                const EmRowX<T> X = em_fetch_x(c, s, t);
                const EmB<T> B = em_bvals(c, W);
                const cx<T> ex1_t = W.ex1[1];
                em_step<T, IO_RING_G>(c, sp, W, B, t, p0, p1, row_inv(c, t), X, ring);
                if (t == g.nr - 1) em_ghost_bth<T, IO_RING_G>(c, sp, W, B, p1, ring);
                if (t >= 0 && t < g.nr) {
                    cx<T> f[NS];
                    sa_factors(a, m, W, B, ex1_t, f);
#pragma unroll
                    for (int q = 0; q < NS; ++q) put(q, f[q]);
                    sa_row = true;
                }
            }
            __syncthreads();
            if (sa_row) sa_store(t, a.sa);
            __syncthreads();
        }
    } else {
        SetP<T> s2 = s;    // the second step's extra currents
        s2.jxa = s.jxb; s2.jra = s.jrb; s2.jta = s.jtb;
        cx<T> xa_pre = em_xa(c, s2, jsc);
        cx<T> xa_nxt = em_xa(c, s2, jsc + 1);
        EmRowX<T> xrt = em_xrt(c, s2, jsc);
        for (int t = jsp; t <= jec + 2; ++t) {
            const int j = t - 2;
            bool sa_row = false;
            if (j == jsc - 1) {
                if (jsc >= 0) em_take(c, W, em_fetch_ring(c, ring, jsc, xa_pre), jsc, g.nr);
            } else if (j >= jsc && j <= jec) {
                em_rotate(W);
                em_take(c, W, em_fetch_ring(c, ring, j + 1, xa_nxt), j + 1, g.nr);
                const EmRowX<T> X = em_fetch_x_ring(c, ring, j, xrt);
                if (j < jec) {
                    xa_nxt = em_xa(c, s2, j + 2);
                    xrt = em_xrt(c, s2, j + 1);
                }
                const EmB<T> B = em_bvals(c, W);
                const cx<T> ex1_j = W.ex1[1];
                em_step<T, IO_FROM_RING>(c, s2, W, B, j, r0, r1, row_inv(c, j), X, ring);
                if (j == g.nr - 1) em_ghost_bth<T, IO_FROM_RING>(c, s2, W, B, r1, ring);
                if (j >= 0 && j < g.nr) {
                    cx<T> f[NS];
                    sa_factors(a, m, W, B, ex1_j, f);
#pragma unroll
                    for (int q = 0; q < NS; ++q) put(q, f[q]);
                    sa_row = true;
                }
            }
            __syncthreads();
            if (sa_row) sa_store(j, a.sa2);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// batched launches: block -> (instance, tile) through the launch's list; the
// instance's arguments are read from a device table
// ---------------------------------------------------------------------------
template <typename T, int M, bool AXT>
__device__ __forceinline__ void batch_a_body(const FusedArgs<T>* __restrict__ args, const BatchList& L) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int k = batch_find(L, b);
    const FusedArgs<T>& a = args[L.idx[k]];
    const int local = b - L.first[k];
    // strips fastest: the tiles an XCD runs together are neighbouring strips of
    // one radial chunk, which share the cache lines at their edges (measured 8%
    // faster for the FP64 step than radial chunks fastest)
    const int strips = fused_strips(a.g.nx);
    fused_a_body<T, M, AXT>(a, local % strips, local / strips, L.rows);
}
template <int M, bool AXT>
__global__ void __launch_bounds__(WAVE * M) k_batch_a_f64(const FusedArgs<double>* __restrict__ args, BatchList L) {
    batch_a_body<double, M, AXT>(args, L);
}
template <int M, bool AXT>
__global__ void __launch_bounds__(WAVE * M) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_a_f32(const FusedArgs<float>* __restrict__ args, BatchList L) {
    batch_a_body<float, M, AXT>(args, L);
}

template <typename T, int M>
__device__ __forceinline__ void batch_ax_body(const FusedArgs<T>* __restrict__ args, const BatchList& L) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int k = batch_find(L, b);
    const FusedArgs<T>& a = args[L.idx[k]];
    const int local = b - L.first[k];
    const int strips = fused_strips(a.g.nx);   // strips fastest, as kernel A
    fused_ax_body<T, M>(a, local % strips, local / strips, L.rows);
}
template <typename T, int M>
__global__ void __launch_bounds__(WAVE * M) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_ax(const FusedArgs<T>* __restrict__ args, BatchList L) {
    batch_ax_body<T, M>(args, L);
}

template <typename T, int WHICH>
__global__ void __launch_bounds__(WAVE) k_batch_em(const FusedArgs<T>* __restrict__ args, BatchList L) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int k = batch_find(L, b);
    const FusedArgs<T>& a = args[L.idx[k]];
    const int local = b - L.first[k];
    const int chunks = (a.g.nr + 1 + L.rows - 1) / L.rows;
    const int m = local % a.g.M;                 // the modes of one tile run side by side
    const int t = local / a.g.M;
    em_body<T, WHICH>(a, t / chunks, t % chunks, m, L.rows);
}

template <typename T, int M>
__global__ void __launch_bounds__(2 * WAVE * M) k_batch_a2(const FusedArgs<T>* __restrict__ args, BatchList L) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int k = batch_find(L, b);
    const FusedArgs<T>& a = args[L.idx[k]];
    const int local = b - L.first[k];
    const int strips = pair_strips(a.g.nx);   // strips fastest, as kernel A
    fused_a2_body<T, M>(a, local % strips, local / strips, L.rows);
}

template <typename T, int WHICH, int PL>
__global__ void __launch_bounds__(2 * WAVE) k_batch_em2(const FusedArgs<T>* __restrict__ args, BatchList L) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int k = batch_find(L, b);
    const FusedArgs<T>& a = args[L.idx[k]];
    const int local = b - L.first[k];
    const int chunks = (a.g.nr + 1 + L.rows - 1) / L.rows;
    const int m = local % a.g.M;                 // the modes of one tile run side by side
    const int t = local / a.g.M;
    em2_body<T, WHICH, PL>(a, t / chunks, t % chunks, m, L.rows);
}

}  // namespace fused

template <typename T>
hipError_t drive_plane(const Drive& d, const Geo& g, cx<T>* out, cx<T>* out2, int64_t n, int64_t w, int64_t dw,
                       hipStream_t s) {
    hipLaunchKernelGGL((fused::k_drive_plane<T>),
                       dim3((g.nx + 255) / 256, (g.nr + fused::kDriveRows) / fused::kDriveRows, out2 ? 2 : 1), dim3(256), 0,
                       s, d, g, out, out2, n, w, dw);
    return hipGetLastError();
}

// Raises a kernel's dynamic LDS limit once per process (needed above 64 KiB:
// the exchange buffers of kernel A at 6 or more modes in FP64).
static hipError_t allow_lds(const void* kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
}

template <typename T, bool AXT>
static hipError_t batch_a_mode(const FusedArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s) {
    const size_t lds = 2 * size_t(fused::NS) * M * fused::WAVE * sizeof(cx<T>);
    switch (M) {
#define QDS_BA(MM)                                                                                                      \
    case MM:                                                                                                            \
        if constexpr (sizeof(T) == 8) {                                                                                 \
            static const hipError_t attr = allow_lds(reinterpret_cast<const void*>(&fused::k_batch_a_f64<MM, AXT>), lds); \
            if (attr != hipSuccess) return attr;                                                                        \
            hipLaunchKernelGGL((fused::k_batch_a_f64<MM, AXT>), dim3(blocks), dim3(fused::WAVE * MM), lds, s, args, L); \
        } else {                                                                                                        \
            static const hipError_t attr = allow_lds(reinterpret_cast<const void*>(&fused::k_batch_a_f32<MM, AXT>), lds); \
            if (attr != hipSuccess) return attr;                                                                        \
            hipLaunchKernelGGL((fused::k_batch_a_f32<MM, AXT>), dim3(blocks), dim3(fused::WAVE * MM), lds, s, args, L); \
        }                                                                                                               \
        break;
        QDS_BA(1) QDS_BA(2) QDS_BA(3) QDS_BA(4) QDS_BA(5) QDS_BA(6) QDS_BA(7) QDS_BA(8)
#undef QDS_BA
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t batch_a(const FusedArgs<T>* args, const BatchList& L, int M, int blocks, bool axt, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    return axt ? batch_a_mode<T, true>(args, L, M, blocks, s) : batch_a_mode<T, false>(args, L, M, blocks, s);
}

template <typename T>
hipError_t batch_ax(const FusedArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    const size_t lds = size_t(fused::NS + fused::NJ) * M * fused::WAVE * sizeof(cx<T>);
    switch (M) {
#define QDS_BX(MM)                                                                                     \
    case MM: {                                                                                         \
        /* above 64 KiB of LDS per workgroup (FP64, three or four modes) */                            \
        static const hipError_t attr = hipFuncSetAttribute(                                            \
            reinterpret_cast<const void*>(&fused::k_batch_ax<T, MM>),                                  \
            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));                                     \
        if (attr != hipSuccess) return attr;                                                           \
        hipLaunchKernelGGL((fused::k_batch_ax<T, MM>), dim3(blocks), dim3(fused::WAVE * MM), lds, s, args, L); \
        break;                                                                                         \
    }
        QDS_BX(1) QDS_BX(2) QDS_BX(3) QDS_BX(4)
#undef QDS_BX
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t batch_em(const FusedArgs<T>* args, const BatchList& L, int which, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (which)
        hipLaunchKernelGGL((fused::k_batch_em<T, 1>), dim3(blocks), dim3(fused::WAVE), 0, s, args, L);
    else
        hipLaunchKernelGGL((fused::k_batch_em<T, 0>), dim3(blocks), dim3(fused::WAVE), 0, s, args, L);
    return hipGetLastError();
}

// the instantiation of the two-step march for (which, plasma)
template <typename T>
static auto em2_kernel(int which, bool plasma) {
    return which ? (plasma ? fused::k_batch_em2<T, 1, 1> : fused::k_batch_em2<T, 1, 0>)
                 : (plasma ? fused::k_batch_em2<T, 0, 1> : fused::k_batch_em2<T, 0, 0>);
}

template <typename T>
hipError_t batch_em2(const FusedArgs<T>* args, const BatchList& L, int which, bool plasma, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    const size_t lds = size_t(fused::RG_N) * fused::RING_ROWS * fused::WAVE * sizeof(cx<T>);
    hipLaunchKernelGGL(em2_kernel<T>(which, plasma), dim3(blocks), dim3(2 * fused::WAVE), lds, s, args, L);
    return hipGetLastError();
}

template <typename T>
int em2_blocks_per_cu(int which, bool plasma) {
    const size_t lds = size_t(fused::RG_N) * fused::RING_ROWS * fused::WAVE * sizeof(cx<T>);
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, em2_kernel<T>(which, plasma), 2 * fused::WAVE, lds);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

size_t a2_lds_bytes(int M, size_t elem_bytes) {
    return size_t(M) * (size_t(fused::RG_N) * fused::RING_ROWS + 2 * fused::NS) * fused::WAVE * 2 * elem_bytes;
}

template <typename T>
hipError_t batch_a2(const FusedArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    const size_t lds = a2_lds_bytes(M, sizeof(T));
    switch (M) {
#define QDS_BA2(MM)                                                                                       \
    case MM: {                                                                                            \
        static const hipError_t attr = allow_lds(reinterpret_cast<const void*>(&fused::k_batch_a2<T, MM>), lds); \
        if (attr != hipSuccess) return attr;                                                              \
        hipLaunchKernelGGL((fused::k_batch_a2<T, MM>), dim3(blocks), dim3(2 * fused::WAVE * MM), lds, s, args, L); \
        break;                                                                                            \
    }
        QDS_BA2(1) QDS_BA2(2) QDS_BA2(3) QDS_BA2(4)
#undef QDS_BA2
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t batch_a<double>(const FusedArgs<double>*, const BatchList&, int, int, bool, hipStream_t);
template hipError_t batch_a<float>(const FusedArgs<float>*, const BatchList&, int, int, bool, hipStream_t);
template hipError_t batch_ax<double>(const FusedArgs<double>*, const BatchList&, int, int, hipStream_t);
template hipError_t batch_ax<float>(const FusedArgs<float>*, const BatchList&, int, int, hipStream_t);
template hipError_t batch_em<double>(const FusedArgs<double>*, const BatchList&, int, int, hipStream_t);
template hipError_t batch_em<float>(const FusedArgs<float>*, const BatchList&, int, int, hipStream_t);
template hipError_t batch_em2<double>(const FusedArgs<double>*, const BatchList&, int, bool, int, hipStream_t);
template hipError_t batch_em2<float>(const FusedArgs<float>*, const BatchList&, int, bool, int, hipStream_t);
template int em2_blocks_per_cu<double>(int, bool);
template int em2_blocks_per_cu<float>(int, bool);
template hipError_t batch_a2<double>(const FusedArgs<double>*, const BatchList&, int, int, hipStream_t);
template hipError_t batch_a2<float>(const FusedArgs<float>*, const BatchList&, int, int, hipStream_t);
template hipError_t drive_plane<double>(const Drive&, const Geo&, cx<double>*, cx<double>*, int64_t, int64_t, int64_t,
                                        hipStream_t);
template hipError_t drive_plane<float>(const Drive&, const Geo&, cx<float>*, cx<float>*, int64_t, int64_t, int64_t,
                                       hipStream_t);

}  // namespace qds
