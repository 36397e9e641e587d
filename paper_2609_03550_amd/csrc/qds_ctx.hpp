// Host-side handle of libqds and the helpers shared by its C ABI sources.
#pragma once
#include <stdio.h>

#include <vector>

#include "../../include/qds.h"
#include "qds_kernels.hpp"

struct qds_ctx {
    qds_grid g;
    int M;
    double h;
    double mu_half;          // largest eigenvalue of the half-row radial operator (Klein-Gordon bound)
    int ld;
    size_t plane_elems;      // complex elements per plane
    size_t elem_bytes;       // 16 (F64) or 8 (F32)
    int slot[QDS_NPLANES];   // plane -> position in the buffer, -1 if absent
    int nplanes;
    void* scratch;           // axion-current planes (3) and S_a, library owned
    void* drive_plane;       // j_x^(0) of the prescribed drive, mode 0, for two steps (allocated on first use)
    void* psrc;              // particle currents at the source points, 3 planes (allocated on first use)
    void* pairbuf;           // pairs of steps with the regenerated set: a state-sized buffer for the
                             // background set and axion between the two steps, then j_a (3 planes)
                             // and S_a (1 plane) of the second step; allocated on first use
    int path;                // QDS_PATH_*
    int theta;               // QDS_PRODUCTS_THETA: theta-grid products (staged path)
    int rows;                // the last QDS_OPT_ROWS value (also copied into trows)
    int trows[4];            // tile heights of the table-driven kernels: A, current, B, two-step march
    int tune;                // autotune the tile heights on the next long enough qds_step
    int tuned;
    int timing;              // record per-kernel HIP events in qds_step
    int overlap;             // kernel A of step k+1 on a second stream beside kernel B of step k
    int kernel_ax;           // 1: one-pass kernel AX instead of kernel A and the marched axion kernel
    int pair;                // 1: advance steps in pairs with the two-step march of one set where it applies
    int pair_a;              // 1: in pairs, the background set too by its two-step march with the axion source
    hipStream_t side;        // that stream (created on first use, default priority)
    hipEvent_t ev_x, ev_a;   // its ordering events
    // timing events, recorded without synchronising and resolved by
    // qds_get_timing: pairs (start, end) per launch, tagged with the kernel
    std::vector<hipEvent_t> pool;
    size_t used;
    std::vector<int> tag;
    // kernel argument table of the fused kernels (device copy, pinned host
    // staging and the event that marks the end of its last upload)
    void* ktab_dev;
    void* ktab_pin;
    size_t ktab_bytes;
    hipEvent_t ktab_ev;
    bool ktab_valid;
    double ktab_key[18];     // buffers and physics the uploaded table was built for
    char err[256];
};

namespace qdsi {

inline thread_local char g_err[256] = "";

// Event pair for the next timed launch (created on demand, reused after a reset).
inline hipEvent_t* timing_pair(qds_ctx* c, int kernel) {
    if (c->used + 2 > c->pool.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            c->pool.push_back(e);
        }
    }
    hipEvent_t* p = &c->pool[c->used];
    c->used += 2;
    c->tag.push_back(kernel);
    return p;
}

inline qds_status fail(qds_ctx* c, qds_status s, const char* fmt, const char* detail = "") {
    char* buf = c ? c->err : g_err;
    snprintf(buf, 256, fmt, detail);
    return s;
}

inline bool has(const qds_ctx* c, int plane) { return c->slot[plane] >= 0; }

// Bytes of the pair buffer: a state, then j_a (3 planes) and S_a (1 plane) of
// a pair's second step.
inline size_t pairbuf_bytes(const qds_ctx* c) {
    return (size_t(c->nplanes) + 4) * c->plane_elems * c->elem_bytes;
}

template <typename T>
void plane_table(const qds_ctx* c, void* base, qds::cx<T>** out) {
    for (int p = 0; p < QDS_NPLANES; ++p) {
        out[p] = c->slot[p] < 0 ? nullptr
                                : reinterpret_cast<qds::cx<T>*>(static_cast<char*>(base) +
                                                                size_t(c->slot[p]) * c->plane_elems * c->elem_bytes);
    }
}

inline qds::Geo geo(const qds_ctx* c) {
    qds::Geo g;
    g.nx = c->g.nx;
    g.nr = c->g.nr;
    g.M = c->M;
    g.ld = c->ld;
    g.h = c->h;
    g.dr = c->g.dr;
    g.per = c->g.x_bc == QDS_X_PERIODIC;
    g.open_r = c->g.r_bc == QDS_R_OPEN;
    return g;
}

// The fused kernels cover up to 8 modes (one wavefront per mode; kernel AX up
// to 4).  With the moving window and the regenerated set, the axion current
// needs the background set's new state at the old state's columns while the
// background march writes it one column left: only kernel AX, which forms the
// current from the values in its registers, takes that combination (up to 4
// modes; beyond, the staged kernels, which shift after the whole step).
inline bool fused_ok(const qds_ctx* c) {
    const bool window_arem = c->g.x_bc == QDS_X_WINDOW && (c->g.content & QDS_HAS_AREM);
    // the fused kernels address a plane with 32-bit byte offsets
    const bool small_planes = c->plane_elems * c->elem_bytes < (size_t(1) << 32);
    return c->M <= 8 && (!window_arem || c->M <= 4) && small_planes;
}

inline bool use_fused(const qds_ctx* c) {
    if (c->path == QDS_PATH_STAGED || c->theta) return false;
    return fused_ok(c);
}

template <typename T>
qds::SetP<T> fused_set(qds::cx<T>* const* A, qds::cx<T>* const* B, int s) {
    const int b = 9 * s;
    qds::SetP<T> p;
    p.trp = A[b + 0]; p.trm = A[b + 1]; p.ttp = A[b + 2]; p.ttm = A[b + 3];
    p.ex = A[b + 4]; p.bx = A[b + 5]; p.jx = A[b + 6]; p.jr = A[b + 7]; p.jt = A[b + 8];
    p.otrp = B[b + 0]; p.otrm = B[b + 1]; p.ottp = B[b + 2]; p.ottm = B[b + 3];
    p.oex = B[b + 4]; p.obx = B[b + 5]; p.ojx = B[b + 6]; p.ojr = B[b + 7]; p.ojt = B[b + 8];
    p.jxa = p.jra = p.jta = nullptr;
    p.jxb = p.jrb = p.jtb = nullptr;
    p.jxa_m0 = 0;
    return p;
}

template <typename T>
qds::StepPlan<T> make_plan(const qds_ctx* c, const qds_current* J, const qds_axion* ax) {
    qds::StepPlan<T> p;
    p.g = geo(c);
    p.plasma = has(c, QDS_P_JX);
    p.axion = has(c, QDS_P_PHI);
    p.arem = has(c, QDS_P_SET1);
    p.theta = c->theta;
    p.wp2 = J ? J->wp2 : 0.0;
    if (!p.plasma) p.wp2 = 0.0;
    p.ma2 = ax ? ax->ma2 : 0.0;
    p.s_phi = ax ? ax->s_phi : 1.0;
    p.s_j = ax ? ax->s_j : 1.0;
    p.bx0 = ax ? qds::cx<T>{T(ax->bext[0]), T(ax->bext[1])} : qds::cx<T>{T(0), T(0)};
    p.br1 = ax ? qds::cx<T>{T(ax->bext[2]), T(ax->bext[3])} : qds::cx<T>{T(0), T(0)};
    p.bt1 = ax ? qds::cx<T>{T(ax->bext[4]), T(ax->bext[5])} : qds::cx<T>{T(0), T(0)};
    p.drive.on = (J && J->kind == QDS_J_RING) ? 1 : 0;
    if (p.drive.on) {
        p.drive.amp = J->amp; p.drive.x0 = J->x0; p.drive.v = J->v; p.drive.sx = J->sx;
        p.drive.r0 = J->r0; p.drive.sr = J->sr; p.drive.noise = J->noise; p.drive.seed = J->seed;
    }
    // scratch planes: j_a,x, j_a,r, j_a,theta, S_a
    qds::cx<T>* sc[4];
    for (int k = 0; k < 4; ++k)
        sc[k] = c->scratch ? reinterpret_cast<qds::cx<T>*>(static_cast<char*>(c->scratch) +
                                                           size_t(k) * c->plane_elems * c->elem_bytes)
                           : nullptr;
    for (int k = 0; k < 3; ++k) p.ja[k] = sc[k];
    p.sa = sc[3];
    // j_a of the second step of a pair: the 3 planes after the pair buffer's state
    const size_t sbytes = size_t(c->nplanes) * c->plane_elems * c->elem_bytes;
    for (int k = 0; k < 3; ++k)
        p.ja2[k] = c->pairbuf ? reinterpret_cast<qds::cx<T>*>(static_cast<char*>(c->pairbuf) + sbytes +
                                                              size_t(k) * c->plane_elems * c->elem_bytes)
                              : nullptr;
    p.jdrv = static_cast<qds::cx<T>*>(c->drive_plane);
    p.jdrv2 = c->drive_plane ? reinterpret_cast<qds::cx<T>*>(static_cast<char*>(c->drive_plane) +
                                                            size_t(c->g.nr + 1) * size_t(c->ld) * c->elem_bytes)
                             : nullptr;
    const bool part = J && J->kind == QDS_J_PARTICLES;
    p.pj[0] = part ? static_cast<qds::cx<T>*>(const_cast<void*>(J->pjx_prev)) : nullptr;
    p.pj[1] = part ? static_cast<qds::cx<T>*>(const_cast<void*>(J->pjx_next)) : nullptr;
    p.pj[2] = part ? static_cast<qds::cx<T>*>(const_cast<void*>(J->pjr)) : nullptr;
    p.pj[3] = part ? static_cast<qds::cx<T>*>(const_cast<void*>(J->pjt)) : nullptr;
    p.psrc[0] = p.psrc[1] = p.psrc[2] = nullptr;   // set where the fused kernels take them
    return p;
}

// Whether T_a and phi move from kernel A to the marched axion current, which
// then advances them from the S_a that kernel A leaves in scratch (with the
// regenerated set; the fused kernels do not take it with the moving window).
template <typename T>
bool march_axion(const qds_ctx* c, const qds::StepPlan<T>& p0) {
    return p0.axion && p0.arem && c->g.x_bc != QDS_X_WINDOW && p0.sa != nullptr;
}

// Whether one launch of kernel AX advances the background set, the axion and
// the axion current together: with the regenerated set, up to 4 modes, when
// QDS_OPT_KERNEL_AX asks for it or the moving window needs it.
template <typename T>
bool fuse_ax(const qds_ctx* c, const qds::StepPlan<T>& p0) {
    if (!(p0.axion && p0.arem && p0.sa != nullptr) || c->M > 4) return false;
    return c->kernel_ax || c->g.x_bc == QDS_X_WINDOW;
}

// Fused-kernel arguments of one step from buffer A (old) to buffer B (new).
// With a prescribed drive the background set reads the drive plane, which
// holds j_x^(0) of the step, as its extra j_x of mode 0.
template <typename T>
qds::FusedArgs<T> fused_args(const qds_ctx* c, const qds::StepPlan<T>& p0, void* bufA, void* bufB) {
    qds::FusedArgs<T> a{};
    a.g = p0.g;
    a.plasma = p0.plasma;
    a.axion = p0.axion;
    a.wp2 = p0.wp2; a.ma2 = p0.ma2; a.s_phi = p0.s_phi; a.s_j = p0.s_j;
    a.bx0 = p0.bx0; a.br1 = p0.br1; a.bt1 = p0.bt1;
    a.window = c->g.x_bc == QDS_X_WINDOW;
    a.jax = p0.ja[0]; a.jar = p0.ja[1]; a.jat = p0.ja[2];
    a.sa = march_axion(c, p0) ? p0.sa : nullptr;
    qds::cx<T>* A[QDS_NPLANES];
    qds::cx<T>* B[QDS_NPLANES];
    plane_table<T>(c, bufA, A);
    plane_table<T>(c, bufB, B);
    a.s0 = fused_set<T>(A, B, 0);
    a.s1 = fused_set<T>(A, B, 1);
    a.s1.jxa = a.jax; a.s1.jra = a.jar; a.s1.jta = a.jat;
    a.s1.jxb = p0.ja2[0]; a.s1.jrb = p0.ja2[1]; a.s1.jtb = p0.ja2[2];
    if (p0.drive.on) {
        a.s0.jxa = p0.jdrv;
        a.s0.jxa_m0 = 1;
    }
    if (p0.psrc[0]) {
        // particle currents at the source points, every mode
        a.s0.jxa = p0.psrc[0];
        a.s0.jra = p0.psrc[1];
        a.s0.jta = p0.psrc[2];
        a.s0.jxa_m0 = 0;
    }
    // a pair of steps of the background set alone (no drive) reads the same
    // extra currents in both steps
    if (!p0.drive.on) {
        a.s0.jxb = a.s0.jxa; a.s0.jrb = a.s0.jra; a.s0.jtb = a.s0.jta;
    } else {
        a.s0.jxb = p0.jdrv2;   // j_x^(0) of the pair's second step
    }
    a.phi = A[QDS_P_PHI]; a.tap = A[QDS_P_TAP]; a.tam = A[QDS_P_TAM];
    a.ophi = B[QDS_P_PHI]; a.otap = B[QDS_P_TAP]; a.otam = B[QDS_P_TAM];
    return a;
}

// Whether qds_step advances steps in pairs, with the two-step march of one
// set: the regenerated set (kernel A and the marched axion kernel for the
// background set and the axion; no prescribed drive, no moving window), or
// the background set alone (no axion; with or without the prescribed drive
// and the moving window).
template <typename T>
bool pair_ok(const qds_ctx* c, const qds::StepPlan<T>& p0) {
    if (!c->pair) return false;
    if (p0.arem) return march_axion(c, p0) && !fuse_ax(c, p0) && !p0.drive.on;
    return !p0.axion;
}

// Whether a pair of steps also advances the background set by its two-step
// march with the axion source (in place of kernel A twice): QDS_OPT_PAIR_A,
// the regenerated set in pairs, up to 4 modes, and its LDS within a CU.
template <typename T>
bool pair_a2(const qds_ctx* c, const qds::StepPlan<T>& p0) {
    return c->pair_a && pair_ok(c, p0) && p0.arem && c->M <= 4 &&
           qds::a2_lds_bytes(c->M, c->elem_bytes / 2) <= 160 * 1024;
}

// Axion-current arguments of the same step.
template <typename T>
qds::AxionArgs<T> axion_args(const qds_ctx* c, const qds::StepPlan<T>& p0, void* bufA, void* bufB) {
    qds::StepPlan<T> pl = p0;
    plane_table<T>(c, bufA, pl.A);
    plane_table<T>(c, bufB, pl.B);
    qds::AxionArgs<T> x = pl.axion_args();
    x.sa = march_axion(c, p0) ? p0.sa : nullptr;
    return x;
}

inline qds_status check_state(qds_ctx* c, const qds_state* st) {
    if (!st) return fail(c, QDS_EINVAL, "null state%s");
    if (!st->buf[0] || !st->buf[1] || st->buf[0] == st->buf[1])
        return fail(c, QDS_ESTATE, "state needs two distinct device buffers%s");
    if (st->cur != 0 && st->cur != 1) return fail(c, QDS_ESTATE, "state.cur must be 0 or 1%s");
    if (st->step < 0 || st->window < 0) return fail(c, QDS_ESTATE, "negative step or window%s");
    if (st->step >= (int64_t(1) << 31)) return fail(c, QDS_ESTATE, "step counter out of range%s");
    return QDS_OK;
}

// Argument table of the fused kernels for one handle: entry q is the step that
// reads state buffer q and writes buffer 1 - q; single-entry launch lists.
template <typename T>
struct KTab {
    qds::FusedArgs<T> fa[2];
    qds::AxionArgs<T> xa[2];
    // a pair of steps from buffer q: [q][0] the background set and the axion
    // from buffer q into the pair buffer (j_a into the first j_a planes),
    // [q][1] from the pair buffer into buffer 1 - q (j_a into the second);
    // the two-step march of the regenerated set uses fa[q]
    qds::FusedArgs<T> fp[2][2];
    qds::AxionArgs<T> xp[2][2];
    // with the background set's two-step march: its arguments (buffer q to
    // buffer 1 - q, the first step's field planes and the second S_a in the
    // pair buffer) and those of the second axion kernel (reading that S_a)
    qds::FusedArgs<T> fa2[2];
    qds::AxionArgs<T> xp2[2];
    int idx[2];
    int firstA[2], firstC[2], firstB[2], firstB2[2], firstA2[2];
};

}  // namespace qdsi
