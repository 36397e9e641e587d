// Kernel argument blocks and host-side entry points of the QDS step.
#pragma once
#include "qds_common.hpp"

namespace qds {

// Axis reflections (Sec. 2.3 regularity).  A scalar or longitudinal mode m
// (B_x, phi, T_a) behaves as r^m near the axis: its ghost at r_{-1/2} is
// (-1)^m times the value at r_{1/2}.  A transverse component (E_r, B_theta,
// T_r) of mode m behaves as r^|m-1|: parity (-1)^(m-1) for m != 1, while mode
// 1 takes the axis relation ghost = 2i T_theta(0) - T_r(1/2); tghost is the
// coefficient of T_r(1/2) in either.
template <typename T>
__device__ __forceinline__ T parity(int m) { return (m & 1) ? T(-1) : T(1); }
template <typename T>
__device__ __forceinline__ T tghost(int m) { return (m & 1) && m != 1 ? T(1) : T(-1); }

// Grid geometry and plane addressing: element (mode m, row, column c) of a
// plane is at (m * (nr + 1) + row) * ld + c.
struct Geo {
    int nx, nr, M, ld;
    double h, dr;
    int per;      // periodic x
    int open_r;   // outflow at r = R_max (else conducting wall)
    __host__ __device__ __forceinline__ size_t at(int m, int row, int c) const {
        return (size_t(m) * size_t(nr + 1) + size_t(row)) * size_t(ld) + size_t(c);
    }
};

struct Drive {
    int on;
    double amp, x0, v, sx, r0, sr, noise;
    uint64_t seed;
};

template <typename T>
struct SetPtr {
    cx<T>* trp;
    cx<T>* trm;
    cx<T>* ttp;
    cx<T>* ttm;
    cx<T>* ex;
    cx<T>* bx;
    cx<T>* jx;   // plasma planes (null without plasma)
    cx<T>* jr;
    cx<T>* jt;
};

template <typename T>
struct StageArgs {
    Geo g;
    SetPtr<T> A, B;             // old / new state of this set
    const cx<T>* jx_add;        // extra currents at the source points (or null)
    const cx<T>* jr_add;
    const cx<T>* jt_add;
    // particle currents of the background set (deposits of the PIC coupling):
    // j_x at (x_{i+1/2}, r_j) from the steps ending at t^{n-1/2} and t^{n+1/2}
    // (j_x^n is their mean; either may be null), j_r and j_theta at t^{n+1/2}
    // on integer columns (averaged here to x_{i+1/2}); null when absent
    const cx<T>* pjx0;
    const cx<T>* pjx1;
    const cx<T>* pjr;
    const cx<T>* pjt;
    int plasma;
    double wp2;
    Drive drive;                // prescribed j_x^(0) (background set only)
    int64_t n, w;               // step and window offset
};

template <typename T>
struct AxionArgs {
    Geo g;
    SetPtr<T> A0, B0;           // background set, old / new
    const cx<T>* phiA;
    const cx<T>* tapA;
    const cx<T>* tamA;
    cx<T>* phiB;
    cx<T>* tapB;
    cx<T>* tamB;
    cx<T>* jax;                 // scratch: axion current at the source points
    cx<T>* jar;
    cx<T>* jat;
    // scratch S_a (kernel A's output) when the marched current kernel also
    // advances T_a and phi; null when kernel A does
    const cx<T>* sa;
    double ma2, s_phi, s_j;
    cx<T> bx0, br1, bt1;        // uniform external field (B_x^(0), B_r^(1), B_theta^(1))
};

// Everything one step needs: two state buffers (old A, new B) as plane
// pointer tables, the physics and the step counters.
template <typename T>
struct StepPlan {
    Geo g;
    cx<T>* A[21];
    cx<T>* B[21];
    cx<T>* ja[3];
    cx<T>* ja2[3];              // j_a of the second step of a pair of steps (null until used)
    cx<T>* sa;                  // scratch S_a plane (regenerated set only)
    cx<T>* jdrv;                // drive plane (j_x^(0) of mode 0; null until first used)
    cx<T>* jdrv2;               // the drive plane of the second step of a pair
    int plasma, axion, arem;
    int theta;                  // staged path: theta-grid products instead of the direct convolution
    double wp2, ma2, s_phi, s_j;
    cx<T> bx0, br1, bt1;
    Drive drive;
    const cx<T>* pj[4];         // particle currents of set 0 (StageArgs::pjx0 ..), or null
    cx<T>* psrc[3];             // the same at the source points (fused kernels), or null
    int64_t n, w;

    SetPtr<T> set(cx<T>* const* P, int s) const {
        const int b = 9 * s;
        return SetPtr<T>{P[b + 0], P[b + 1], P[b + 2], P[b + 3], P[b + 4], P[b + 5], P[b + 6], P[b + 7], P[b + 8]};
    }
    StageArgs<T> set_args(int s) const {
        StageArgs<T> a;
        a.g = g;
        a.A = set(A, s);
        a.B = set(B, s);
        a.jx_add = s ? ja[0] : nullptr;
        a.jr_add = s ? ja[1] : nullptr;
        a.jt_add = s ? ja[2] : nullptr;
        a.plasma = plasma;
        a.wp2 = wp2;
        a.drive = drive;
        if (s) a.drive.on = 0;
        a.pjx0 = s ? nullptr : pj[0];
        a.pjx1 = s ? nullptr : pj[1];
        a.pjr = s ? nullptr : pj[2];
        a.pjt = s ? nullptr : pj[3];
        a.n = n;
        a.w = w;
        return a;
    }
    AxionArgs<T> axion_args() const {
        AxionArgs<T> x;
        x.g = g;
        x.A0 = set(A, 0);
        x.B0 = set(B, 0);
        x.phiA = A[18]; x.tapA = A[19]; x.tamA = A[20];
        x.phiB = B[18]; x.tapB = B[19]; x.tamB = B[20];
        x.jax = ja[0]; x.jar = ja[1]; x.jat = ja[2];
        x.sa = nullptr;
        x.ma2 = ma2; x.s_phi = s_phi; x.s_j = s_j;
        x.bx0 = bx0; x.br1 = br1; x.bt1 = bt1;
        return x;
    }
};

// One electromagnetic set for the fused kernels: old planes, new planes and
// the extra currents at the source points (regenerated set only).
template <typename T>
struct SetP {
    const cx<T>* trp; const cx<T>* trm; const cx<T>* ttp; const cx<T>* ttm;
    const cx<T>* ex; const cx<T>* bx; const cx<T>* jx; const cx<T>* jr; const cx<T>* jt;
    cx<T>* otrp; cx<T>* otrm; cx<T>* ottp; cx<T>* ottm;
    cx<T>* oex; cx<T>* obx; cx<T>* ojx; cx<T>* ojr; cx<T>* ojt;
    const cx<T>* jxa; const cx<T>* jra; const cx<T>* jta;
    // the extra currents of the following step, read by the second step of
    // the two-step march (the axion current of that step; null when absent)
    const cx<T>* jxb; const cx<T>* jrb; const cx<T>* jtb;
    int jxa_m0;   // jxa holds mode 0 only (the prescribed drive); other modes add nothing
};

template <typename T>
struct FusedArgs {
    Geo g;
    SetP<T> s0, s1;
    const cx<T>* phi; const cx<T>* tap; const cx<T>* tam;
    cx<T>* ophi; cx<T>* otap; cx<T>* otam;
    cx<T>* jax; cx<T>* jar; cx<T>* jat;   // axion current scratch
    // non-null: kernel A writes the axion source S_a here (unshifted columns,
    // no moving window) and leaves T_a and phi to the axion-current march
    cx<T>* sa;
    // the background set's two-step march with the axion source: the first
    // step's field planes (T^+-, E_x, B_x, what the axion kernel reads) and
    // the second step's S_a
    cx<T>* mtrp; cx<T>* mtrm; cx<T>* mttp; cx<T>* mttm; cx<T>* mex; cx<T>* mbx;
    cx<T>* sa2;
    int plasma, axion;
    double wp2, ma2, s_phi, s_j;
    cx<T> bx0, br1, bt1;
    int window;       // 1: moving window (outputs one column to the left)
};

// Columns owned by one 64-lane strip of the r-marching kernels: lane 0 is the
// left halo, lanes 62 and 63 the right halo (lane 63 only lends its column).
constexpr int kFusedOwn = 61;
__host__ __device__ inline int fused_strips(int nx) { return (nx + kFusedOwn - 1) / kFusedOwn; }
// The two-step march of one set: its second step needs the first step's
// results on lanes k-1 .. k+2, so a strip owns 58 columns (lanes 2-59).
constexpr int kPairOwn = 58;
__host__ __device__ inline int pair_strips(int nx) { return (nx + kPairOwn - 1) / kPairOwn; }
// With the moving window the second step's strips start one column further
// left, so one more column must be covered.
__host__ __device__ inline int pair_strips(int nx, int window) { return pair_strips(nx + window); }

// One launch of a batched kernel: the instances it covers (indices into the
// argument tables), the first block of each (n + 1 entries, first[0] = 0, the
// last is the grid size) and the tile height in rows.
struct BatchList {
    const int* idx;
    const int* first;
    int n;
    int rows;
};

// Tile of block b of a launch of n blocks.  Workgroups are dispatched to the
// 8 XCDs round-robin (block b on XCD b % 8); this gives each XCD a contiguous
// run of tiles, so tiles that share halo rows and columns run on one L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b & 7, k = b >> 3;
    const int q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + k;
}

// Instance of tile b: the largest k with first[k] <= b.
__device__ __forceinline__ int batch_find(const BatchList& L, int b) {
    int lo = 0, hi = L.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.first[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T> hipError_t staged_step(const StepPlan<T>& p, hipStream_t s);
// Particle deposits (Sec. 3.1) brought to the source points where the
// background set takes its currents: j_x^n = (j_x^{n-1/2} + j_x^{n+1/2})/2 at
// x_{i+1/2} (pjx0 may be null), and j_r, j_theta of the step ending at
// t^{n+1/2} averaged from x_i, x_{i+1} to x_{i+1/2}; written to the three
// planes of out (the layout of a state plane).
template <typename T>
hipError_t particle_sources(const cx<T>* pjx0, const cx<T>* pjx1, const cx<T>* pjr, const cx<T>* pjt, const Geo& g,
                            cx<T>* out, size_t plane_elems, hipStream_t s);
// The prescribed drive's j_x^(0) of step n (window offset w) into the mode-0
// rows of out (one plane of row pitch g.ld), read by the background set of the
// fused kernels as its extra j_x; with out2, in the same launch, that of step
// n + 1 (window offset w + dw) into out2.
template <typename T>
hipError_t drive_plane(const Drive& d, const Geo& g, cx<T>* out, cx<T>* out2, int64_t n, int64_t w, int64_t dw,
                       hipStream_t s);
// Batched launches over many instances (argument tables in device memory).
// axt: kernel A advances the axion (every instance of the list has sa null);
// otherwise every instance has sa set and the axion current advances it.
template <typename T>
hipError_t batch_a(const FusedArgs<T>* args, const BatchList& L, int M, int blocks, bool axt, hipStream_t s);
template <typename T>
hipError_t batch_em(const FusedArgs<T>* args, const BatchList& L, int which, int blocks, hipStream_t s);
// Two steps of one set in one pass (set 1 with the axion currents s1.jxa/jra/jta
// of the first step and s1.jxb/jrb/jtb of the second; set 0 without an axion):
// reads the set from the A planes and writes it, two steps on, to the B planes.
// Tiles of pair_strips(nx) strips x rows-high chunks x modes, 128 threads each.
// plasma false: no instance of the list carries plasma currents (a leaner
// instantiation).
template <typename T>
hipError_t batch_em2(const FusedArgs<T>* args, const BatchList& L, int which, bool plasma, int blocks, hipStream_t s);
// Workgroups of that launch of the two-step march that one CU holds at once,
// as the runtime computes it from the kernel's registers and ring; 0 if it
// cannot tell.
template <typename T>
int em2_blocks_per_cu(int which, bool plasma);
// Two steps of the background set with the axion source of each (2M waves per
// tile of pair_strips(nx) strips x rows-high chunks): reads s0's A planes,
// writes the first step's field planes to mtrp..mbx and its S_a to sa, the
// second step's state to s0's B planes and its S_a to sa2.  LDS: M x 48 KiB
// in FP64, M x 24 KiB in FP32 (a2_lds_bytes), at most 160 KiB.
template <typename T>
hipError_t batch_a2(const FusedArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s);
size_t a2_lds_bytes(int M, size_t elem_bytes);
// Kernel AX: the background set, the axion source, the axion advance and the
// axion current in one launch (every instance of the list has sa set).
template <typename T>
hipError_t batch_ax(const FusedArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s);
template <typename T>
hipError_t batch_current(const AxionArgs<T>* args, const BatchList& L, int M, int blocks, hipStream_t s);
// Column strips of the marching axion-current kernel (61 owned columns each,
// as kernel A).
int current_strips(int nx);
// One transposed step.  march: the axion-current transpose marches in r
// (needs planes below 4 GiB); otherwise one thread per cell with atomic adds.
template <typename T>
hipError_t adjoint_step(const StepPlan<T>& p, cx<T>* const* Ab, cx<T>* const* Bb, cx<T>* const* jab, double* dLds,
                        bool march, hipStream_t s);
template <typename T>
hipError_t loss_seed(cx<T>* const* U, cx<T>* const* Ub, const Geo& g, int set, int md, int x0, int x1, double* loss,
                     hipStream_t s);
template <typename T> hipError_t dot(const void* a, const void* b, size_t n, double* out, hipStream_t s);
template <typename T> hipError_t window_shift(const cx<T>* src, cx<T>* dst, const Geo& g, int nplanes, hipStream_t s);
template <typename T>
hipError_t add_pulse(SetPtr<T> s0, const Geo& g, int pol, const double* fK, const double* fJ, const double* fG,
                     hipStream_t s);

}  // namespace qds
