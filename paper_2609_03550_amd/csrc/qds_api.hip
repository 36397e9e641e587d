// C ABI of libqds (declared in include/qds.h): validation, handle, plane
// layout and the per-step launch sequence.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "qds_ctx.hpp"

using namespace qdsi;

namespace {

// Tile-height candidates of the autotuner (two passes over four per kernel
// class): kernel A (the background set with the axion), kernel AX (the
// background set, the axion and its current in one pass), the marched axion
// kernel, kernel B (the regenerated set), and the background set alone, whose
// one-wave tiles want tall chunks on large grids (26 rows fill the GPU once at
// 4096 x 256 x 3) and short ones on small grids.
const int kCandA[4] = {8, 16, 24, 32};
const int kCandAX[4] = {16, 24, 32, 48};
const int kCandCur[4] = {4, 6, 8, 16};
const int kCandB[4] = {16, 32, 52, 64};
const int kCandEm[4] = {8, 16, 26, 52};
const int kCandA2[4] = {16, 24, 32, 43};
// Tile heights of the two-step march.  Its workgroups march their chunks in
// lockstep rounds, and it runs fastest where a launch's workgroups (strips x
// chunks x modes) just fit in a whole number of rounds of what the GPU holds
// at once (measured on MI355X: at 8192 x 256 x 3 all resident at once, 129
// rows in FP64 and 86 in FP32; on the 4096 x 256 x 3 window workload 29 rows,
// just under two rounds, in both).  Candidates: the heights of
// the three smallest distinct chunk counts that fill 1, 2, 3, ... rounds, and
// 20 rows; without an occupancy figure from the runtime, the heights that cut
// the nr + 1 rows into 2, 4 and 3 chunks.
template <typename T>
void cand_pair(const qds_ctx* c, int which, bool plasma, int* out) {
    const int R = c->g.nr + 1;
    const int per = qds::pair_strips(c->g.nx, c->g.x_bc == QDS_X_WINDOW ? 1 : 0) * c->M;   // workgroups per chunk row
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 0;
    }
    const int64_t slots = int64_t(qds::em2_blocks_per_cu<T>(which, plasma)) * cus;
    int chunks[3] = {2, 4, 3};
    if (slots > 0) {
        int n = 0, last = 0;
        for (int64_t k = 1; n < 3 && k <= 64; ++k) {
            const int64_t q = std::min<int64_t>(k * slots / per, R);
            if (q >= 1 && q != last) chunks[n++] = last = int(q);
        }
        for (; n < 3; ++n) chunks[n] = last > 0 ? last : 2;
    }
    for (int q = 0; q < 3; ++q) {
        const int h = (R + chunks[q] - 1) / chunks[q];
        out[q] = h < 4 ? 4 : h;
    }
    out[3] = 20;
}
constexpr int kTrials = 8;

// Makes the device argument table current for the state buffers of st
// (uploaded on the stream only when it changed).
template <typename T>
qds_status sync_ktab(qds_ctx* c, const qds_state* st, const qds::StepPlan<T>& p0, hipStream_t s, KTab<T>** dev) {
    // the table depends on the two buffers, the physics and the tile height only
    double key[18];
    memset(key, 0, sizeof(key));
    memcpy(&key[0], &st->buf[0], sizeof(void*));
    memcpy(&key[1], &st->buf[1], sizeof(void*));
    key[2] = p0.wp2; key[3] = p0.ma2; key[4] = p0.s_phi; key[5] = p0.s_j;
    key[6] = double(p0.bx0.re); key[7] = double(p0.bx0.im); key[8] = double(p0.br1.re); key[9] = double(p0.br1.im);
    key[10] = double(p0.bt1.re); key[11] = double(p0.bt1.im);
    key[12] = double(c->trows[0]); key[13] = double(c->trows[1]); key[14] = double(c->trows[2]);
    key[15] = double(p0.drive.on) + (p0.psrc[0] ? 2.0 : 0.0);
    memcpy(&key[16], &c->pairbuf, sizeof(void*));
    key[17] = double(c->trows[3]);
    if (!c->ktab_dev) {
        c->ktab_bytes = sizeof(KTab<double>);
        if (hipMalloc(&c->ktab_dev, c->ktab_bytes) != hipSuccess) {
            c->ktab_dev = nullptr;
            return fail(c, QDS_ENOMEM, "hipMalloc of the argument table failed%s");
        }
        if (hipHostMalloc(&c->ktab_pin, c->ktab_bytes, hipHostMallocDefault) != hipSuccess) {
            c->ktab_pin = nullptr;
            return fail(c, QDS_ENOMEM, "hipHostMalloc of the argument table failed%s");
        }
        if (hipEventCreateWithFlags(&c->ktab_ev, hipEventDisableTiming) != hipSuccess)
            return fail(c, QDS_EHIP, "event creation failed%s");
        c->ktab_valid = false;
    }
    *dev = static_cast<KTab<T>*>(c->ktab_dev);
    if (c->ktab_valid && memcmp(key, c->ktab_key, sizeof(key)) == 0) return QDS_OK;
    KTab<T> t;
    memset(&t, 0, sizeof(t));
    for (int q = 0; q < 2; ++q) {
        t.fa[q] = fused_args<T>(c, p0, st->buf[q], st->buf[1 - q]);
        t.xa[q] = axion_args<T>(c, p0, st->buf[q], st->buf[1 - q]);
        if (c->pairbuf) {
            // the second step of a pair writes its axion current to the second j_a planes
            qds::StepPlan<T> p2 = p0;
            for (int k = 0; k < 3; ++k) p2.ja[k] = p0.ja2[k];
            t.fp[q][0] = fused_args<T>(c, p0, st->buf[q], c->pairbuf);
            t.xp[q][0] = axion_args<T>(c, p0, st->buf[q], c->pairbuf);
            t.fp[q][1] = fused_args<T>(c, p2, c->pairbuf, st->buf[1 - q]);
            t.xp[q][1] = axion_args<T>(c, p2, c->pairbuf, st->buf[1 - q]);
            // the background set's two-step march: the first step's field
            // planes into the pair buffer, the second S_a after its j_a planes
            qds::cx<T>* P[QDS_NPLANES];
            plane_table<T>(c, c->pairbuf, P);
            qds::cx<T>* sa2 = p0.ja2[2] + c->plane_elems;
            t.fa2[q] = fused_args<T>(c, p0, st->buf[q], st->buf[1 - q]);
            t.fa2[q].mtrp = P[QDS_P_TRP]; t.fa2[q].mtrm = P[QDS_P_TRM];
            t.fa2[q].mttp = P[QDS_P_TTP]; t.fa2[q].mttm = P[QDS_P_TTM];
            t.fa2[q].mex = P[QDS_P_EX]; t.fa2[q].mbx = P[QDS_P_BX];
            t.fa2[q].sa2 = sa2;
            qds::StepPlan<T> p3 = p2;
            p3.sa = sa2;
            t.xp2[q] = axion_args<T>(c, p3, c->pairbuf, st->buf[1 - q]);
        }
    }
    const int strips = qds::fused_strips(c->g.nx);
    auto chunks = [&](int rows) { return (c->g.nr + 1 + rows - 1) / rows; };
    t.idx[0] = t.idx[1] = 0;
    t.firstA[1] = strips * chunks(c->trows[0]);
    t.firstC[1] = qds::current_strips(c->g.nx) * chunks(c->trows[1]);
    t.firstB[1] = strips * chunks(c->trows[2]) * c->M;
    t.firstB2[1] = qds::pair_strips(c->g.nx, c->g.x_bc == QDS_X_WINDOW ? 1 : 0) * chunks(c->trows[3]) * c->M;
    t.firstA2[1] = qds::pair_strips(c->g.nx) * chunks(c->trows[0]);
    // the staging copy may still be read by the previous upload
    if (c->ktab_valid && hipEventSynchronize(c->ktab_ev) != hipSuccess)
        return fail(c, QDS_EHIP, "argument table upload failed%s");
    memcpy(c->ktab_pin, &t, sizeof(t));
    hipError_t e = hipMemcpyAsync(c->ktab_dev, c->ktab_pin, sizeof(t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(c, QDS_EHIP, "argument table upload failed: %s", hipGetErrorString(e));
    e = hipEventRecord(c->ktab_ev, s);
    if (e != hipSuccess) return fail(c, QDS_EHIP, "argument table upload failed: %s", hipGetErrorString(e));
    memcpy(c->ktab_key, key, sizeof(key));
    c->ktab_valid = true;
    return QDS_OK;
}

// Device view of one step's entry in an argument table: the kernel
// arguments, the single-entry launch lists and their block counts.
template <typename T>
struct TabView {
    const qds::FusedArgs<T>* fa;
    const qds::AxionArgs<T>* xa;
    const int* idx;
    const int* firstA;
    const int* firstC;
    const int* firstB;
    const int* firstB2;
    const int* firstA2;
    int nA, nC, nB, nB2, nA2;
};

template <typename T>
TabView<T> ktab_view(KTab<T>* K, const KTab<T>& host, int q) {
    return TabView<T>{K->fa + q, K->xa + q, K->idx, K->firstA, K->firstC, K->firstB, K->firstB2, K->firstA2,
                      host.firstA[1], host.firstC[1], host.firstB[1], host.firstB2[1], host.firstA2[1]};
}

// The three launches of one fused step through an argument-table entry:
// kernel A (or the background set alone), the axion kernel and the
// regenerated set, each on stream s and bracketed by the event pair e when
// given (or by a timing pair when timing is on).
enum { kLaunchA = 0, kLaunchX = 1, kLaunchB = 2, kLaunchB2 = 3, kLaunchA2 = 4 };

template <typename T>
qds_status table_launch_one(qds_ctx* c, const qds::StepPlan<T>& p0, const TabView<T>& v, int which, hipStream_t s,
                            hipEvent_t* e) {
    auto list = [&](const int* first_dev, int rows) {
        qds::BatchList L;
        L.idx = v.idx;
        L.first = first_dev;
        L.n = 1;
        L.rows = rows;
        return L;
    };
    // timing slots: 0 kernel A (or the background set alone, also its
    // two-step march), 1 the regenerated set (also its two-step march), 2 the
    // axion kernel
    const int slot = (which == kLaunchA || which == kLaunchA2)
                         ? 0
                         : (which == kLaunchX ? 2 : (which == kLaunchB2 && !p0.arem ? 0 : 1));
    hipEvent_t* ev = e ? e : (c->timing ? timing_pair(c, slot) : nullptr);
    if (ev && hipEventRecord(ev[0], s) != hipSuccess) return fail(c, QDS_EHIP, "event record failed%s");
    hipError_t err = hipSuccess;
    if (which == kLaunchA) {
        if (fuse_ax(c, p0)) {
            err = qds::batch_ax<T>(v.fa, list(v.firstA, c->trows[0]), c->M, v.nA, s);
        } else if (p0.axion) {
            err = qds::batch_a<T>(v.fa, list(v.firstA, c->trows[0]), c->M, v.nA, !march_axion(c, p0), s);
        } else {
            // the background set alone: the kernel-B march with the kernel-A tile
            const int strips = qds::fused_strips(c->g.nx);
            err = qds::batch_em<T>(v.fa, list(v.firstB, c->trows[0]), 0,
                                   strips * ((c->g.nr + c->trows[0]) / c->trows[0]) * c->M, s);
        }
    } else if (which == kLaunchX) {
        err = qds::batch_current<T>(v.xa, list(v.firstC, c->trows[1]), c->M, v.nC, s);
    } else if (which == kLaunchB2) {
        err = qds::batch_em2<T>(v.fa, list(v.firstB2, c->trows[3]), p0.arem ? 1 : 0, p0.plasma != 0, v.nB2, s);
    } else if (which == kLaunchA2) {
        err = qds::batch_a2<T>(v.fa, list(v.firstA2, c->trows[0]), c->M, v.nA2, s);
    } else {
        err = qds::batch_em<T>(v.fa, list(v.firstB, c->trows[2]), 1, v.nB, s);
    }
    if (err != hipSuccess) return fail(c, QDS_EHIP, "launch failed: %s", hipGetErrorString(err));
    if (ev && hipEventRecord(ev[1], s) != hipSuccess) return fail(c, QDS_EHIP, "event record failed%s");
    return QDS_OK;
}

// One fused step (kernel A or the background set, then the axion current
// and the regenerated set), each launch bracketed by the event pair
// ev[2k], ev[2k+1] when ev is given.
template <typename T>
qds_status table_launch(qds_ctx* c, const qds::StepPlan<T>& p0, const TabView<T>& v, hipStream_t s, hipEvent_t* ev) {
    qds_status r = table_launch_one<T>(c, p0, v, kLaunchA, s, ev);
    if (r != QDS_OK || !p0.arem) return r;
    if (!fuse_ax(c, p0) && (r = table_launch_one<T>(c, p0, v, kLaunchX, s, ev ? ev + 2 : nullptr)) != QDS_OK)
        return r;
    return table_launch_one<T>(c, p0, v, kLaunchB, s, ev ? ev + 4 : nullptr);
}

template <typename T>
qds_status table_step(qds_ctx* c, qds_state* st, const qds::StepPlan<T>& p0, KTab<T>* K, const KTab<T>& host,
                      hipStream_t s, hipEvent_t* ev) {
    if (p0.drive.on) {
        // this step's j_x^(0), read by the background set as its extra j_x
        const hipError_t e = qds::drive_plane<T>(p0.drive, p0.g, p0.jdrv, nullptr, st->step, st->window, 0, s);
        if (e != hipSuccess) return fail(c, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    }
    const qds_status r = table_launch<T>(c, p0, ktab_view<T>(K, host, st->cur), s, ev);
    if (r != QDS_OK) return r;
    st->cur = 1 - st->cur;
    if (c->g.x_bc == QDS_X_WINDOW) st->window += 1;
    st->step += 1;
    return QDS_OK;
}

// Two steps from buffer q to buffer 1 - q.  With the regenerated set: kernel
// A and the axion kernel of the first step write the background set and the
// axion to the pair buffer (the axion current to the first j_a planes), those
// of the second step from there to buffer 1 - q (the axion current to the
// second j_a planes), then the two-step march takes the regenerated set from
// buffer q to buffer 1 - q with both currents.  Without it the two-step march
// of the background set is the only launch.  The event pairs ev[0..1] (first
// kernel A), ev[2..3] (first axion kernel) and ev[4..5] (the two-step march)
// bracket those launches when ev is given.
template <typename T>
qds_status pair_step(qds_ctx* c, qds_state* st, const qds::StepPlan<T>& p0, KTab<T>* K, const KTab<T>& host,
                     hipStream_t s, hipEvent_t* ev) {
    const int q = st->cur;
    const TabView<T> v = ktab_view<T>(K, host, q);
    const bool window = c->g.x_bc == QDS_X_WINDOW;
    qds_status r;
    if (p0.drive.on) {
        // j_x^(0) of both steps (the second one column on with the window)
        const hipError_t e =
            qds::drive_plane<T>(p0.drive, p0.g, p0.jdrv, p0.jdrv2, st->step, st->window, window ? 1 : 0, s);
        if (e != hipSuccess) return fail(c, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    }
    if (p0.arem && pair_a2(c, p0)) {
        // the background set's two-step march, then the axion kernel of each step
        TabView<T> va = v, vb = v;
        va.fa = &K->fa2[q]; va.xa = &K->xp[q][0];
        vb.xa = &K->xp2[q];
        if ((r = table_launch_one<T>(c, p0, va, kLaunchA2, s, ev)) != QDS_OK) return r;
        if ((r = table_launch_one<T>(c, p0, va, kLaunchX, s, ev ? ev + 2 : nullptr)) != QDS_OK) return r;
        if ((r = table_launch_one<T>(c, p0, vb, kLaunchX, s, nullptr)) != QDS_OK) return r;
    } else if (p0.arem) {
        TabView<T> va = v, vb = v;
        va.fa = &K->fp[q][0]; va.xa = &K->xp[q][0];
        vb.fa = &K->fp[q][1]; vb.xa = &K->xp[q][1];
        if ((r = table_launch_one<T>(c, p0, va, kLaunchA, s, ev)) != QDS_OK) return r;
        if ((r = table_launch_one<T>(c, p0, va, kLaunchX, s, ev ? ev + 2 : nullptr)) != QDS_OK) return r;
        if ((r = table_launch_one<T>(c, p0, vb, kLaunchA, s, nullptr)) != QDS_OK) return r;
        if ((r = table_launch_one<T>(c, p0, vb, kLaunchX, s, nullptr)) != QDS_OK) return r;
    }
    if ((r = table_launch_one<T>(c, p0, v, kLaunchB2, s, ev ? ev + 4 : nullptr)) != QDS_OK) return r;
    st->cur = 1 - st->cur;
    st->step += 2;
    if (window) st->window += 2;
    return QDS_OK;
}

// Steps with kernel A of step k+1 running on a second stream beside kernel B
// of step k.  A(k+1) reads and writes the background set and S_a; B(k) reads
// the regenerated set and j_a and writes the regenerated set: they share no
// plane.  A(k+1) waits for the axion kernel of step k (the last reader of
// S_a and of the background buffer A(k+1) overwrites); the axion kernel of
// step k+1 waits for A(k+1) and, on the caller's stream, for B(k) (the reader
// of the j_a it overwrites).  Every side-stream launch is joined back into
// the caller's stream before the call returns.
template <typename T>
qds_status overlapped_steps(qds_ctx* c, qds_state* st, const qds::StepPlan<T>& p0, KTab<T>* K, const KTab<T>& host,
                            int64_t n, hipStream_t s) {
    if (!c->side) {
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
            c->side = nullptr;
            return fail(c, QDS_EHIP, "side stream creation failed%s");
        }
        if (hipEventCreateWithFlags(&c->ev_x, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_a, hipEventDisableTiming) != hipSuccess)
            return fail(c, QDS_EHIP, "event creation failed%s");
    }
    qds_status r = table_launch_one<T>(c, p0, ktab_view<T>(K, host, st->cur), kLaunchA, s, nullptr);
    if (r != QDS_OK) return r;
    for (int64_t k = 0; k < n; ++k) {
        const TabView<T> v = ktab_view<T>(K, host, st->cur);
        if ((r = table_launch_one<T>(c, p0, v, kLaunchX, s, nullptr)) != QDS_OK) return r;
        const bool more = k + 1 < n;
        if (more) {
            if (hipEventRecord(c->ev_x, s) != hipSuccess || hipStreamWaitEvent(c->side, c->ev_x, 0) != hipSuccess)
                return fail(c, QDS_EHIP, "stream ordering failed%s");
            // the next step reads the buffer this step writes
            if ((r = table_launch_one<T>(c, p0, ktab_view<T>(K, host, 1 - st->cur), kLaunchA, c->side, nullptr)) !=
                QDS_OK)
                return r;
            if (hipEventRecord(c->ev_a, c->side) != hipSuccess) return fail(c, QDS_EHIP, "event record failed%s");
        }
        if ((r = table_launch_one<T>(c, p0, v, kLaunchB, s, nullptr)) != QDS_OK) return r;
        st->cur = 1 - st->cur;
        st->step += 1;
        if (more && hipStreamWaitEvent(s, c->ev_a, 0) != hipSuccess) return fail(c, QDS_EHIP, "stream ordering failed%s");
    }
    return QDS_OK;
}

template <typename T>
qds_status fused_steps(qds_ctx* c, qds_state* st, const qds::StepPlan<T>& p1, int64_t n_steps, hipStream_t s) {
    KTab<T>* K;
    qds_status r;
    int64_t done = 0;
    qds::StepPlan<T> p0 = p1;
    if (p0.drive.on && !c->drive_plane) {
        // the drive planes (mode 0 of one plane, for the two steps of a pair),
        // allocated on first use
        if (hipMalloc(&c->drive_plane, 2 * size_t(c->g.nr + 1) * size_t(c->ld) * c->elem_bytes) != hipSuccess) {
            c->drive_plane = nullptr;
            return fail(c, QDS_ENOMEM, "hipMalloc of the drive plane failed%s");
        }
    }
    p0.jdrv = static_cast<qds::cx<T>*>(c->drive_plane);
    p0.jdrv2 = c->drive_plane ? reinterpret_cast<qds::cx<T>*>(static_cast<char*>(c->drive_plane) +
                                                             size_t(c->g.nr + 1) * size_t(c->ld) * c->elem_bytes)
                              : nullptr;
    if (p0.pj[1]) {
        // particle deposits: the background march reads them at the source
        // points, formed once per call (they hold for every step of it)
        const size_t pb = c->plane_elems * c->elem_bytes;
        if (!c->psrc && hipMalloc(&c->psrc, 3 * pb) != hipSuccess) {
            c->psrc = nullptr;
            return fail(c, QDS_ENOMEM, "hipMalloc of the particle source planes failed%s");
        }
        for (int k = 0; k < 3; ++k)
            p0.psrc[k] = reinterpret_cast<qds::cx<T>*>(static_cast<char*>(c->psrc) + size_t(k) * pb);
        const hipError_t e = qds::particle_sources<T>(p0.pj[0], p0.pj[1], p0.pj[2], p0.pj[3], p0.g, p0.psrc[0],
                                                      c->plane_elems, s);
        if (e != hipSuccess) return fail(c, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    }
    const bool pairs = pair_ok(c, p0) && n_steps >= 2;
    if (pairs && p0.arem && !c->pairbuf) {
        // the background set and the axion between the two steps of a pair,
        // then the second step's axion current and axion source
        if (hipMalloc(&c->pairbuf, pairbuf_bytes(c)) != hipSuccess) {
            c->pairbuf = nullptr;
            return fail(c, QDS_ENOMEM, "hipMalloc of the pair buffer failed%s");
        }
    }
    if (c->pairbuf) {
        // (the plan was made before the buffer existed on the first call)
        const size_t sbytes = size_t(c->nplanes) * c->plane_elems * c->elem_bytes;
        for (int k = 0; k < 3; ++k)
            p0.ja2[k] = reinterpret_cast<qds::cx<T>*>(static_cast<char*>(c->pairbuf) + sbytes +
                                                      size_t(k) * c->plane_elems * c->elem_bytes);
    }
    const int per = pairs ? 2 : 1;     // steps per trial
    if (c->tune && n_steps >= per * kTrials) {
        // autotuner: timed ordinary steps (or pairs of steps), two passes over
        // four tile heights per kernel (candidates around each kernel's
        // measured optimum).  Slots: 0 kernel A / the background set, 1 the
        // axion kernel, 2 kernel B or the two-step march.
        int candB2[4];
        if (pairs) cand_pair<T>(c, p0.arem ? 1 : 0, p0.plasma != 0, candB2);
        const int* cand[3] = {fuse_ax(c, p0) ? kCandAX
                                             : (pairs && pair_a2(c, p0) ? kCandA2 : (p0.axion ? kCandA : kCandEm)),
                              kCandCur, pairs ? candB2 : kCandB};
        int* const tr[3] = {&c->trows[0], &c->trows[1], pairs ? &c->trows[3] : &c->trows[2]};
        const bool run[3] = {!(pairs && !p0.arem), p0.arem && !fuse_ax(c, p0), p0.arem || pairs};
        std::vector<hipEvent_t> ev(6 * kTrials);
        for (hipEvent_t& x : ev)
            if (hipEventCreate(&x) != hipSuccess) return fail(c, QDS_EHIP, "event creation failed%s");
        for (int t = 0; t < kTrials; ++t) {
            for (int k = 0; k < 3; ++k)
                if (run[k]) *tr[k] = cand[k][t % 4];
            if ((r = sync_ktab<T>(c, st, p0, s, &K)) != QDS_OK) return r;
            const KTab<T> host = *static_cast<const KTab<T>*>(c->ktab_pin);
            r = pairs ? pair_step<T>(c, st, p0, K, host, s, ev.data() + 6 * t)
                      : table_step<T>(c, st, p0, K, host, s, ev.data() + 6 * t);
            if (r != QDS_OK) return r;
        }
        if (hipStreamSynchronize(s) != hipSuccess) return fail(c, QDS_EHIP, "tuning steps failed%s");
        // fastest trial of each candidate; for the bandwidth-bound marches of
        // the sets (slots 0 and 2), among the candidates within the trials'
        // noise (2%) of the fastest, the tallest, whose chunks re-read the
        // fewest halo rows; for the axion kernel, whose time is set by its
        // workgroups in flight rather than its bytes, the fastest
        float best[3][4];
        for (int k = 0; k < 3; ++k)
            for (int q = 0; q < 4; ++q) best[k][q] = 3.4e38f;
        for (int t = 0; t < kTrials; ++t)
            for (int k = 0; k < 3; ++k) {
                if (!run[k]) continue;
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[6 * t + 2 * k], ev[6 * t + 2 * k + 1]) != hipSuccess) {
                    (void)hipGetLastError();   // do not leave the error for the next launch check
                    continue;
                }
                best[k][t % 4] = std::min(best[k][t % 4], ms);
            }
        for (hipEvent_t x : ev) (void)hipEventDestroy(x);
        for (int k = 0; k < 3; ++k) {
            if (!run[k]) continue;
            float fastest = 3.4e38f;
            for (int q = 0; q < 4; ++q) fastest = std::min(fastest, best[k][q]);
            if (!(fastest < 3.4e38f)) continue;   // no trial timed: keep the last height
            const float tol = k == 1 ? 1.0f : 1.02f;
            int pick = 0;
            for (int q = 0; q < 4; ++q)
                if (best[k][q] <= tol * fastest && (pick == 0 || cand[k][q] > pick)) pick = cand[k][q];
            *tr[k] = pick;
        }
        c->tune = 0;
        c->tuned = 1;
        done = per * kTrials;
    }
    if ((r = sync_ktab<T>(c, st, p0, s, &K)) != QDS_OK) return r;
    const KTab<T> host = *static_cast<const KTab<T>*>(c->ktab_pin);
    if (c->overlap && p0.arem && march_axion(c, p0) && !fuse_ax(c, p0) && !p0.drive.on && c->g.x_bc != QDS_X_WINDOW &&
        n_steps - done >= 2)
        return overlapped_steps<T>(c, st, p0, K, host, n_steps - done, s);
    if (pairs)
        for (; n_steps - done >= 2; done += 2)
            if ((r = pair_step<T>(c, st, p0, K, host, s, nullptr)) != QDS_OK) return r;
    for (int64_t it = done; it < n_steps; ++it)
        if ((r = table_step<T>(c, st, p0, K, host, s, nullptr)) != QDS_OK) return r;
    return QDS_OK;
}

template <typename T>
qds_status run_steps(qds_ctx* c, qds_state* st, const qds_current* J, const qds_axion* ax, int64_t n_steps,
                     hipStream_t s) {
    qds::StepPlan<T> p = make_plan<T>(c, J, ax);
    // particle currents run on the staged kernels
    if (use_fused(c)) return fused_steps<T>(c, st, p, n_steps, s);
    const bool window = c->g.x_bc == QDS_X_WINDOW;
    for (int64_t it = 0; it < n_steps; ++it) {
        int a = st->cur, b = 1 - st->cur;
        plane_table<T>(c, st->buf[a], p.A);
        plane_table<T>(c, st->buf[b], p.B);
        p.n = st->step;
        p.w = st->window;
        hipEvent_t* ev = c->timing ? timing_pair(c, 0) : nullptr;
        if (ev && hipEventRecord(ev[0], s) != hipSuccess) return fail(c, QDS_EHIP, "event record failed%s");
        hipError_t e = qds::staged_step<T>(p, s);
        if (e != hipSuccess) return fail(c, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
        if (ev && hipEventRecord(ev[1], s) != hipSuccess) return fail(c, QDS_EHIP, "event record failed%s");
        if (window) {
            // the new state (in b) moves one cell left into a
            e = qds::window_shift<T>(reinterpret_cast<const qds::cx<T>*>(st->buf[b]),
                                     reinterpret_cast<qds::cx<T>*>(st->buf[a]), p.g, c->nplanes, s);
            if (e != hipSuccess) return fail(c, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
            st->window += 1;
        } else {
            st->cur = b;
        }
        st->step += 1;
    }
    return QDS_OK;
}


// ---------------------------------------------------------------------------
// radial stability bound (the factorised dispersion relation of the scheme)
// ---------------------------------------------------------------------------
// With c dt = dx the one-step map of a mode factorises (periodic x, closed r)
// as sin^2(w dt/2) = sin^2(k dx/2) + (dt/2)^2 mu cos^2(k dx/2) with mu an
// eigenvalue of the discrete radial operator of E_x (integer rows) or B_x
// (half rows), so the step is stable iff dt^2 mu_max <= 4.  Both operators
// are conservative three-point fluxes,
//   (-L F)_j = [c_{j+1/2} (F_j - F_{j+1}) + c_{j-1/2} (F_j - F_{j-1})] / w_j + m^2 F_j / r_j^2,
// symmetric in the inner product sum w_j F_j G_j: E_x rows w_j = r_j (dr/8 on
// the axis), c_{j+1/2} = r_{j+1/2} / dr^2, E_x(0) = 0 for m >= 1; B_x rows
// w = r_{k+1/2}, c = r_k / dr^2 (zero on the axis).  Their largest eigenvalue
// is found by bisection with Sturm counts of the symmetrised tridiagonal
// matrix.  The outer row is taken both with and without its exterior flux
// (conducting wall / open ghost) and the larger value kept.  The Klein-Gordon
// operator is the B_x one plus m_a^2.

// number of eigenvalues below x of the symmetric tridiagonal (a, b)
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
    int neg = 0;
    double d = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        d = (a[i] - x) - (i ? b[i - 1] * b[i - 1] / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++neg;
    }
    return neg;
}

double trid_max(const std::vector<double>& w, const std::vector<double>& clo, const std::vector<double>& chi,
                const std::vector<double>& extra) {
    const size_t n = w.size();
    if (n == 0) return 0.0;
    std::vector<double> a(n), b(n > 1 ? n - 1 : 0);
    double hi = 0.0;
    for (size_t j = 0; j < n; ++j) {
        a[j] = (clo[j] + chi[j]) / w[j] + extra[j];
        if (j + 1 < n) b[j] = -chi[j] / sqrt(w[j] * w[j + 1]);
    }
    for (size_t j = 0; j < n; ++j) hi = fmax(hi, a[j] + (j ? fabs(b[j - 1]) : 0.0) + (j + 1 < n ? fabs(b[j]) : 0.0));
    double lo = 0.0;
    hi *= 1.0 + 1e-12;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(a, b, mid) == int(n)) hi = mid;   // every eigenvalue below mid
        else lo = mid;
    }
    return hi;
}

// mu_max over modes 0..M-1 of the electromagnetic operators (E_x rows, B_x
// rows) and of the Klein-Gordon operator (phi rows, without m_a^2).  A
// conducting wall has E_x(nr) = 0 (a zero neighbour), no flux of E_theta
// through r_nr for B_x, and a zero exterior phi; the open boundary takes the
// larger value with and without the outer row's exterior flux.
void radial_mu_max(int nr, double dr, int M, bool pec, double* mu_em, double* mu_kg) {
    double em = 0.0, kg = 0.0;
    std::vector<double> w, clo, chi, ex;
    auto reset = [&]() { w.clear(); clo.clear(); chi.clear(); ex.clear(); };
    for (int m = 0; m < M; ++m) {
        for (int outer = 0; outer < 2; ++outer) {
            if (pec && outer == 0) continue;   // one exact variant per operator below
            // E_x rows (the axis row only for m = 0; E_x(nr) = 0 at a wall)
            reset();
            const int jend = pec ? nr - 1 : nr;
            for (int j = (m == 0 ? 0 : 1); j <= jend; ++j) {
                w.push_back(j == 0 ? dr / 8.0 : j * dr);
                clo.push_back(j >= 1 ? (j - 0.5) / dr : 0.0);
                chi.push_back(j < jend || pec || outer ? (j + 0.5) / dr : 0.0);
                ex.push_back(j > 0 ? double(m) * m / ((j * dr) * (j * dr)) : 0.0);
            }
            em = fmax(em, trid_max(w, clo, chi, ex));
            // half rows: B_x (no flux through a wall) and phi (zero exterior ghost at a wall)
            for (int kgop = 0; kgop < 2; ++kgop) {
                reset();
                for (int k = 0; k < nr; ++k) {
                    const double rk = (k + 0.5) * dr;
                    const bool flux = k + 1 < nr || (pec ? kgop == 1 : outer == 1);
                    w.push_back(rk);
                    clo.push_back(k / dr);
                    chi.push_back(flux ? (k + 1) / dr : 0.0);
                    ex.push_back(double(m) * m / (rk * rk));
                }
                const double v = trid_max(w, clo, chi, ex);
                if (kgop == 0) em = fmax(em, v);
                else kg = fmax(kg, v);
            }
        }
    }
    *mu_em = em;
    *mu_kg = kg;
}

// ---------------------------------------------------------------------------
// adjoint driver: forward with checkpoints every C steps, loss seed, then per
// segment (last first) recompute the states and run the transposed steps
// ---------------------------------------------------------------------------
size_t backward_pool_bytes(const qds_ctx* c, int64_t n, int64_t C) {
    const size_t S = size_t(c->nplanes) * c->plane_elems * c->elem_bytes;
    const size_t P = c->plane_elems * c->elem_bytes;
    const size_t nck = size_t((n + C - 1) / C);
    return (nck + size_t(C) + 1 + 2) * S + 3 * P + 256;
}

template <typename T>
qds_status backward_impl(qds_ctx* c, const qds_state* u0, const qds_current* J, const qds_axion* ax,
                         const qds_loss* L, int64_t N, int64_t C, void* pool, void* lambda0, double* dLds_out,
                         double* loss_out, hipStream_t s) {
    const size_t S = size_t(c->nplanes) * c->plane_elems * c->elem_bytes;
    const size_t P = c->plane_elems * c->elem_bytes;
    const size_t nck = size_t((N + C - 1) / C);
    // pool layout: the adjoint state pair, the j_a adjoints and the reductions
    // first, then the segment states and the checkpoints
    char* base = static_cast<char*>(pool);
    char* adjX = base;
    char* adjY = adjX + S;
    char* jab = adjY + S;
    double* red = reinterpret_cast<double*>(jab + 3 * P);
    char* seg = jab + 3 * P + 256;
    char* ck = seg + size_t(C + 1) * S;
    auto at_seg = [&](int64_t k) { return static_cast<void*>(seg + size_t(k) * S); };
    hipError_t e = hipSuccess;
#define QDS_TRY(x)                                                                        \
    do {                                                                                  \
        e = (x);                                                                          \
        if (e != hipSuccess) return fail(c, QDS_EHIP, "backward: %s", hipGetErrorString(e)); \
    } while (0)
    QDS_TRY(hipMemsetAsync(red, 0, 4 * sizeof(double), s));
    // forward with checkpoints (two work buffers at the start of the segment area)
    qds_state W;
    W.buf[0] = at_seg(0);
    W.buf[1] = at_seg(1);
    W.cur = 0;
    W.step = u0->step;
    W.window = 0;
    QDS_TRY(hipMemcpyAsync(W.buf[0], u0->buf[u0->cur], S, hipMemcpyDeviceToDevice, s));
    for (int64_t n = 0; n < N; n += C) {
        // one segment at a time (a pending autotune runs on the first one)
        QDS_TRY(hipMemcpyAsync(ck + size_t(n / C) * S, W.buf[W.cur], S, hipMemcpyDeviceToDevice, s));
        qds_status st = run_steps<T>(c, &W, J, ax, (n + C < N) ? C : N - n, s);
        if (st != QDS_OK) return st;
    }
    // loss and its gradient at step N
    qds::cx<T>* U[QDS_NPLANES];
    qds::cx<T>* Yb[QDS_NPLANES];
    qds::cx<T>* Xb[QDS_NPLANES];
    plane_table<T>(c, W.buf[W.cur], U);
    QDS_TRY(hipMemsetAsync(adjY, 0, S, s));
    plane_table<T>(c, adjY, Yb);
    QDS_TRY(qds::loss_seed<T>(U, Yb, geo(c), L->set, L->mode, L->x_begin, L->x_end, red, s));
    // reverse sweep over the segments
    qds::StepPlan<T> p = make_plan<T>(c, J, ax);
    // argument table of the recomputation: entry k advances segment state k
    // into k + 1 (the segment buffers stay in place for the whole sweep)
    qds::FusedArgs<T>* tab = nullptr;
    qds::AxionArgs<T>* xtab = nullptr;
    KTab<T>* K = nullptr;
    KTab<T> khost;
    if (use_fused(c)) {
        qds_state W2 = W;
        if (sync_ktab<T>(c, &W2, p, s, &K) != QDS_OK) return QDS_EHIP;
        khost = *static_cast<const KTab<T>*>(c->ktab_pin);
        const size_t fb = size_t(C) * sizeof(qds::FusedArgs<T>), xb = size_t(C) * sizeof(qds::AxionArgs<T>);
        std::vector<unsigned char> host(fb + xb, 0);
        auto* hf = reinterpret_cast<qds::FusedArgs<T>*>(host.data());
        auto* hx = reinterpret_cast<qds::AxionArgs<T>*>(host.data() + fb);
        for (int64_t k = 0; k < C; ++k) {
            hf[k] = fused_args<T>(c, p, at_seg(k), at_seg(k + 1));
            hx[k] = axion_args<T>(c, p, at_seg(k), at_seg(k + 1));
        }
        void* dtab = nullptr;
        QDS_TRY(hipMalloc(&dtab, fb + xb));
        e = hipMemcpy(dtab, host.data(), fb + xb, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(dtab);
            return fail(c, QDS_EHIP, "backward: %s", hipGetErrorString(e));
        }
        tab = static_cast<qds::FusedArgs<T>*>(dtab);
        xtab = reinterpret_cast<qds::AxionArgs<T>*>(static_cast<char*>(dtab) + fb);
    }
    struct FreeTab {
        void* p;
        ~FreeTab() {
            if (p) (void)hipFree(p);
        }
    } free_tab{tab};
    qds::cx<T>* jb[3];
    for (int k = 0; k < 3; ++k) jb[k] = reinterpret_cast<qds::cx<T>*>(jab + size_t(k) * P);
    for (int64_t sg = int64_t(nck) - 1; sg >= 0; --sg) {
        const int64_t n0 = sg * C, n1 = (n0 + C < N) ? n0 + C : N;
        QDS_TRY(hipMemcpyAsync(at_seg(0), ck + size_t(sg) * S, S, hipMemcpyDeviceToDevice, s));
        for (int64_t k = 0; k < n1 - n0; ++k) {
            if (tab) {
                // fused kernels through the segment's argument table
                const TabView<T> v{tab + k, xtab + k, K->idx, K->firstA, K->firstC, K->firstB, K->firstB2, K->firstA2,
                                   khost.firstA[1], khost.firstC[1], khost.firstB[1], khost.firstB2[1],
                                   khost.firstA2[1]};
                qds_status st = table_launch<T>(c, p, v, s, nullptr);
                if (st != QDS_OK) return st;
                continue;
            }
            qds_state R;
            R.buf[0] = at_seg(k);
            R.buf[1] = at_seg(k + 1);
            R.cur = 0;
            R.step = u0->step + n0 + k;
            R.window = 0;
            qds_status st = run_steps<T>(c, &R, J, ax, 1, s);
            if (st != QDS_OK) return st;
        }
        for (int64_t k = n1 - n0 - 1; k >= 0; --k) {
            plane_table<T>(c, at_seg(k), p.A);
            plane_table<T>(c, at_seg(k + 1), p.B);
            p.n = u0->step + n0 + k;
            p.w = 0;
            QDS_TRY(hipMemsetAsync(adjX, 0, S, s));
            QDS_TRY(hipMemsetAsync(jab, 0, 3 * P, s));
            plane_table<T>(c, adjX, Xb);
            plane_table<T>(c, adjY, Yb);
            QDS_TRY(qds::adjoint_step<T>(p, Xb, Yb, jb, red + 1, use_fused(c), s));
            char* t = adjX; adjX = adjY; adjY = t;
        }
    }
    QDS_TRY(hipMemcpyAsync(lambda0, adjY, S, hipMemcpyDeviceToDevice, s));
    double host[4];
    QDS_TRY(hipMemcpyAsync(host, red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    QDS_TRY(hipStreamSynchronize(s));
#undef QDS_TRY
    if (loss_out) *loss_out = host[0];
    if (dLds_out) {
        dLds_out[0] = host[1];
        dLds_out[1] = host[2];
    }
    return QDS_OK;
}
}  // namespace

extern "C" {

const char* qds_version(void) { return "qds-mi355x 0.1"; }

qds_status qds_radial_mu_max(int32_t nr, double dr, int32_t modes, int32_t r_bc, double* mu_em, double* mu_kg) {
    if (!mu_em || !mu_kg || nr < 2 || !(dr > 0) || modes < 1 || modes > QDS_MAX_MODES || r_bc < 0 || r_bc > 1)
        return fail(nullptr, QDS_EINVAL, "bad argument%s");
    radial_mu_max(nr, dr, modes, r_bc == QDS_R_PEC, mu_em, mu_kg);
    return QDS_OK;
}

const char* qds_last_error(qds_handle h) { return h ? h->err : g_err; }

qds_status qds_init(const qds_grid* grid, int32_t modes, double dx, double dt, qds_handle* out) {
    if (!grid || !out) return fail(nullptr, QDS_EINVAL, "null argument%s");
    *out = nullptr;
    const qds_grid& g = *grid;
    if (g.nx < 8 || g.nr < 4) return fail(nullptr, QDS_EINVAL, "grid too small (nx >= 8, nr >= 4)%s");
    if (g.nx >= (1 << 20) || g.nr >= 4096) return fail(nullptr, QDS_EINVAL, "grid too large%s");
    if (modes < 1 || modes > QDS_MAX_MODES) return fail(nullptr, QDS_EUNSUPPORTED, "modes must be 1..8%s");
    if (g.dtype != QDS_F64 && g.dtype != QDS_F32) return fail(nullptr, QDS_EINVAL, "bad dtype%s");
    if (g.x_bc < 0 || g.x_bc > 2 || g.r_bc < 0 || g.r_bc > 1) return fail(nullptr, QDS_EINVAL, "bad boundary%s");
    if ((g.content & QDS_HAS_AREM) && !(g.content & QDS_HAS_AXION))
        return fail(nullptr, QDS_EINVAL, "regenerated fields need the axion%s");
    if (!(dx > 0) || !(g.dr > 0)) return fail(nullptr, QDS_EINVAL, "dx and dr must be positive%s");
    // exact one-cell transport needs c dt = dx (Sec. 2.1)
    if (fabs(dt - dx) > 4.0 * (nextafter(dx, 2 * dx) - dx))
        return fail(nullptr, QDS_ECFL, "c dt must equal dx%s");
    // radial stability: dt^2 mu_max <= 4 for the largest eigenvalue of the
    // discrete radial operators (see radial_mu_max)
    double mu_em = 0.0, mu_half = 0.0;
    radial_mu_max(g.nr, g.dr, modes, g.r_bc == QDS_R_PEC, &mu_em, &mu_half);
    if (dt * dt * mu_em > 4.0 * (1.0 + 1e-12))
        return fail(nullptr, QDS_ECFL, "radial stability bound dt^2 mu_max <= 4 fails%s");

    qds_ctx* c = new (std::nothrow) qds_ctx();
    if (!c) return fail(nullptr, QDS_ENOMEM, "out of host memory%s");
    c->g = g;
    c->M = modes;
    c->h = dx;
    c->mu_half = mu_half;
    c->ld = (g.nx + 31) / 32 * 32;
    c->plane_elems = size_t(modes) * size_t(g.nr + 1) * size_t(c->ld);
    c->elem_bytes = g.dtype == QDS_F64 ? 16 : 8;
    for (int p = 0; p < QDS_NPLANES; ++p) c->slot[p] = -1;
    int n = 0;
    auto add_set = [&](int base, bool plasma) {
        for (int k = 0; k < 6; ++k) c->slot[base + k] = n++;
        if (plasma)
            for (int k = 6; k < 9; ++k) c->slot[base + k] = n++;
    };
    const bool plasma = g.content & QDS_HAS_PLASMA;
    add_set(0, plasma);
    if (g.content & QDS_HAS_AREM) add_set(QDS_P_SET1, plasma);
    if (g.content & QDS_HAS_AXION)
        for (int k = QDS_P_PHI; k <= QDS_P_TAM; ++k) c->slot[k] = n++;
    c->nplanes = n;
    c->path = QDS_PATH_AUTO;
    c->rows = 16;
    c->trows[0] = c->trows[1] = c->trows[2] = 16;
    c->trows[3] = (g.nr + 2) / 2;   // two chunks
    c->pair = 1;
    if (g.content & QDS_HAS_AREM) {
        // j_a,x, j_a,r, j_a,theta at the source points and the axion source S_a
        hipError_t e = hipMalloc(&c->scratch, 4 * c->plane_elems * c->elem_bytes);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, QDS_ENOMEM, "hipMalloc of the axion-current scratch failed: %s", hipGetErrorString(e));
        }
        e = hipMemset(c->scratch, 0, 4 * c->plane_elems * c->elem_bytes);
        if (e != hipSuccess) {
            (void)hipFree(c->scratch);
            delete c;
            return fail(nullptr, QDS_EHIP, "clearing the axion-current scratch failed: %s", hipGetErrorString(e));
        }
    }
    *out = c;
    return QDS_OK;
}

size_t qds_state_bytes(qds_handle h) { return h ? size_t(h->nplanes) * h->plane_elems * h->elem_bytes : 0; }

int32_t qds_row_pitch(qds_handle h) { return h ? h->ld : 0; }

int64_t qds_plane_offset(qds_handle h, int32_t plane) {
    if (!h || plane < 0 || plane >= QDS_NPLANES || h->slot[plane] < 0) return -1;
    return int64_t(h->slot[plane]) * int64_t(h->plane_elems * h->elem_bytes);
}

qds_status qds_add_pulse(qds_handle h, qds_state* st, int32_t pol, const double* f_K, const double* f_J,
                         const double* f_G, void* stream) {
    if (!h) return fail(nullptr, QDS_EINVAL, "null handle%s");
    qds_status s = check_state(h, st);
    if (s != QDS_OK) return s;
    if (!f_K || !f_J || !f_G) return fail(h, QDS_EINVAL, "null field sample%s");
    if (pol != 'y' && pol != 'z' && pol != 'r' && pol != 't') return fail(h, QDS_EINVAL, "pol must be y, z, r or t%s");
    if ((pol == 'y' || pol == 'z') && h->M < 2) return fail(h, QDS_EINVAL, "a linear polarisation needs mode 1%s");
    hipError_t e;
    qds::Geo g = geo(h);
    if (h->g.dtype == QDS_F64) {
        qds::cx<double>* P[QDS_NPLANES];
        plane_table<double>(h, st->buf[st->cur], P);
        e = qds::add_pulse<double>(qds::SetPtr<double>{P[0], P[1], P[2], P[3], P[4], P[5], P[6], P[7], P[8]}, g, pol,
                                   f_K, f_J, f_G, hipStream_t(stream));
    } else {
        qds::cx<float>* P[QDS_NPLANES];
        plane_table<float>(h, st->buf[st->cur], P);
        e = qds::add_pulse<float>(qds::SetPtr<float>{P[0], P[1], P[2], P[3], P[4], P[5], P[6], P[7], P[8]}, g, pol,
                                  f_K, f_J, f_G, hipStream_t(stream));
    }
    if (e != hipSuccess) return fail(h, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    return QDS_OK;
}

qds_status qds_step(qds_handle h, qds_state* fields, const qds_current* J, const qds_axion* axion, int64_t n_steps,
                    void* stream) {
    if (!h) return fail(nullptr, QDS_EINVAL, "null handle%s");
    qds_status s = check_state(h, fields);
    if (s != QDS_OK) return s;
    if (n_steps < 0) return fail(h, QDS_EINVAL, "negative step count%s");
    if (J && J->kind != QDS_J_NONE && J->kind != QDS_J_RING && J->kind != QDS_J_PARTICLES)
        return fail(h, QDS_EINVAL, "bad current kind%s");
    if (J && J->kind == QDS_J_PARTICLES && (!J->pjx_next || !J->pjr || !J->pjt))
        return fail(h, QDS_EINVAL, "particle currents need pjx_next, pjr and pjt%s");
    if (J && J->kind == QDS_J_PARTICLES && h->g.x_bc == QDS_X_WINDOW)
        return fail(h, QDS_EUNSUPPORTED, "particle currents take no moving window%s");
    if (J && J->kind == QDS_J_RING && (!(J->sx > 0) || !(J->sr > 0)))
        return fail(h, QDS_EINVAL, "drive widths must be positive%s");
    if (J && J->wp2 != 0.0 && !has(h, QDS_P_JX)) return fail(h, QDS_EINVAL, "plasma response needs the plasma planes%s");
    if (fields->step + n_steps >= (int64_t(1) << 31)) return fail(h, QDS_ESTATE, "step counter would overflow%s");
    // the drive noise is keyed on (step, lab column, row) packed as
    // step << 32 | column << 12 | row: every lab column must stay below 2^20
    if (J && J->kind == QDS_J_RING) {
        const int64_t last_col = int64_t(h->g.nx) - 1 + fields->window +
                                 (h->g.x_bc == QDS_X_WINDOW ? n_steps : int64_t(0));
        if (last_col >= (int64_t(1) << 20))
            return fail(h, QDS_ESTATE, "drive noise counter: lab column would reach 2^20 (window + nx + n_steps)%s");
    }
    // the Klein-Gordon operator adds m_a^2 to the half-row radial operator
    if (axion && has(h, QDS_P_PHI) && h->h * h->h * (h->mu_half + axion->ma2) > 4.0 * (1.0 + 1e-12))
        return fail(h, QDS_ECFL, "axion stability bound dt^2 (mu_max + m_a^2) <= 4 fails%s");
    if (h->g.dtype == QDS_F64) return run_steps<double>(h, fields, J, axion, n_steps, hipStream_t(stream));
    return run_steps<float>(h, fields, J, axion, n_steps, hipStream_t(stream));
}

qds_status qds_set_option(qds_handle h, int32_t key, int64_t value) {
    if (!h) return fail(nullptr, QDS_EINVAL, "null handle%s");
    switch (key) {
        case QDS_OPT_PATH:
            if (value < QDS_PATH_AUTO || value > QDS_PATH_FUSED) return fail(h, QDS_EINVAL, "bad path%s");
            if (value == QDS_PATH_FUSED && !fused_ok(h))
                return fail(h, QDS_EUNSUPPORTED, "fused path needs <= 8 modes and no moving window with the regenerated set%s");
            h->path = int(value);
            return QDS_OK;
        case QDS_OPT_ROWS:
            if (value < 1 || value > 4096) return fail(h, QDS_EINVAL, "rows must be 1..4096%s");
            h->rows = int(value);
            h->trows[0] = h->trows[1] = h->trows[2] = h->trows[3] = int(value);
            return QDS_OK;
        case QDS_OPT_ROWS_A:
        case QDS_OPT_ROWS_CUR:
        case QDS_OPT_ROWS_B:
            if (value < 1 || value > 4096) return fail(h, QDS_EINVAL, "rows must be 1..4096%s");
            h->trows[key - QDS_OPT_ROWS_A] = int(value);
            h->tuned = 0;
            return QDS_OK;
        case QDS_OPT_TUNE:
            h->tune = value ? 1 : 0;
            return QDS_OK;
        case QDS_OPT_OVERLAP:
            h->overlap = value ? 1 : 0;
            return QDS_OK;
        case QDS_OPT_KERNEL_AX:
            h->kernel_ax = value ? 1 : 0;
            return QDS_OK;
        case QDS_OPT_PAIR:
            h->pair = value ? 1 : 0;
            return QDS_OK;
        case QDS_OPT_PAIR_A:
            h->pair_a = value ? 1 : 0;
            return QDS_OK;
        case QDS_OPT_ROWS_PAIR:
            if (value < 1 || value > 4096) return fail(h, QDS_EINVAL, "rows must be 1..4096%s");
            h->trows[3] = int(value);
            h->tuned = 0;
            return QDS_OK;
        case QDS_OPT_PRODUCTS:
            if (value != QDS_PRODUCTS_DIRECT && value != QDS_PRODUCTS_THETA)
                return fail(h, QDS_EINVAL, "products must be QDS_PRODUCTS_DIRECT or QDS_PRODUCTS_THETA%s");
            h->theta = value == QDS_PRODUCTS_THETA ? 1 : 0;
            return QDS_OK;
        case QDS_OPT_TIMING:
            h->timing = value ? 1 : 0;
            h->used = 0;
            h->tag.clear();
            return QDS_OK;
        default:
            return fail(h, QDS_EINVAL, "unknown option%s");
    }
}

qds_status qds_get_timing(qds_handle h, double* ms, int64_t* launches) {
    if (!h || !ms || !launches) return fail(h, QDS_EINVAL, "null argument%s");
    ms[0] = ms[1] = ms[2] = 0.0;
    launches[0] = launches[1] = launches[2] = 0;
    for (size_t q = 0; q < h->tag.size(); ++q) {
        float t = 0.f;
        if (hipEventSynchronize(h->pool[2 * q + 1]) != hipSuccess ||
            hipEventElapsedTime(&t, h->pool[2 * q], h->pool[2 * q + 1]) != hipSuccess)
            return fail(h, QDS_EHIP, "reading the timing events failed%s");
        ms[h->tag[q]] += t;
        launches[h->tag[q]] += 1;
    }
    return QDS_OK;
}

qds_status qds_get_tiles(qds_handle h, int32_t* rows, int32_t* tuned) {
    if (!h || !rows) return fail(h, QDS_EINVAL, "null argument%s");
    for (int k = 0; k < 4; ++k) rows[k] = h->trows[k];
    if (tuned) *tuned = h->tuned;
    return QDS_OK;
}

int32_t qds_uses_fused(qds_handle h) { return h && use_fused(h) ? 1 : 0; }


size_t qds_backward_pool_bytes(qds_handle h, int64_t n_steps, int64_t ckpt_every) {
    if (!h || n_steps < 1 || ckpt_every < 1) return 0;
    return backward_pool_bytes(h, n_steps, ckpt_every);
}

qds_status qds_backward(qds_handle h, const qds_state* u0, const qds_current* J, const qds_axion* axion,
                        const qds_loss* loss, int64_t n_steps, int64_t ckpt_every, void* ckpt_pool,
                        size_t pool_bytes, void* lambda0_out, double* dL_ds_out, double* loss_out, void* stream) {
    if (!h) return fail(nullptr, QDS_EINVAL, "null handle%s");
    qds_status s = check_state(h, u0);
    if (s != QDS_OK) return s;
    if (!loss || !ckpt_pool || !lambda0_out) return fail(h, QDS_EINVAL, "null argument%s");
    if (n_steps < 1 || ckpt_every < 1) return fail(h, QDS_EINVAL, "n_steps and ckpt_every must be >= 1%s");
    if (h->g.x_bc == QDS_X_WINDOW) return fail(h, QDS_EUNSUPPORTED, "the adjoint does not cover the moving window%s");
    if (h->M > 4) return fail(h, QDS_EUNSUPPORTED, "the adjoint covers up to 4 modes%s");
    if (loss->set < 0 || loss->set > 1 || (loss->set == 1 && !has(h, QDS_P_SET1)))
        return fail(h, QDS_EINVAL, "loss set not in the state%s");
    if (loss->mode < 0 || loss->mode >= h->M) return fail(h, QDS_EINVAL, "loss mode out of range%s");
    if (loss->x_begin < 0 || loss->x_end > h->g.nx || loss->x_begin >= loss->x_end)
        return fail(h, QDS_EINVAL, "loss column range must satisfy 0 <= x_begin < x_end <= nx%s");
    if (J && J->kind != QDS_J_NONE) return fail(h, QDS_EUNSUPPORTED, "the adjoint has no prescribed drive%s");
    if (pool_bytes < backward_pool_bytes(h, n_steps, ckpt_every))
        return fail(h, QDS_EINVAL, "checkpoint pool too small (see qds_backward_pool_bytes)%s");
    if (u0->step + n_steps >= (int64_t(1) << 31)) return fail(h, QDS_ESTATE, "step counter would overflow%s");
    if (h->g.dtype == QDS_F64)
        return backward_impl<double>(h, u0, J, axion, loss, n_steps, ckpt_every, ckpt_pool, lambda0_out, dL_ds_out,
                                     loss_out, hipStream_t(stream));
    return backward_impl<float>(h, u0, J, axion, loss, n_steps, ckpt_every, ckpt_pool, lambda0_out, dL_ds_out,
                                loss_out, hipStream_t(stream));
}

qds_status qds_dot(qds_handle h, const void* a, const void* b, double* out_dev, void* stream) {
    if (!h || !a || !b || !out_dev) return fail(h, QDS_EINVAL, "null argument%s");
    const size_t n = size_t(h->nplanes) * h->plane_elems;
    hipError_t e = h->g.dtype == QDS_F64 ? qds::dot<double>(a, b, n, out_dev, hipStream_t(stream))
                                         : qds::dot<float>(a, b, n, out_dev, hipStream_t(stream));
    if (e != hipSuccess) return fail(h, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    return QDS_OK;
}


qds_status qds_loss_eval(qds_handle h, const void* buf, const qds_loss* loss, double* out_dev, void* grad_buf,
                         void* stream) {
    if (!h || !buf || !loss || !out_dev) return fail(h, QDS_EINVAL, "null argument%s");
    if (loss->set < 0 || loss->set > 1 || (loss->set == 1 && !has(h, QDS_P_SET1)))
        return fail(h, QDS_EINVAL, "loss set not in the state%s");
    if (loss->mode < 0 || loss->mode >= h->M) return fail(h, QDS_EINVAL, "loss mode out of range%s");
    if (loss->x_begin < 0 || loss->x_end > h->g.nx || loss->x_begin >= loss->x_end)
        return fail(h, QDS_EINVAL, "loss column range must satisfy 0 <= x_begin < x_end <= nx%s");
    hipError_t e;
    const size_t S = size_t(h->nplanes) * h->plane_elems * h->elem_bytes;
    if (!grad_buf) {
        // a scratch gradient buffer is needed by the seed kernel
        void* tmp = nullptr;
        if (hipMallocAsync(&tmp, S, hipStream_t(stream)) != hipSuccess) return fail(h, QDS_ENOMEM, "no memory%s");
        grad_buf = tmp;
        qds_status st = qds_loss_eval(h, buf, loss, out_dev, grad_buf, stream);
        (void)hipFreeAsync(tmp, hipStream_t(stream));
        return st;
    }
    if (h->g.dtype == QDS_F64) {
        qds::cx<double>* U[QDS_NPLANES];
        qds::cx<double>* G[QDS_NPLANES];
        plane_table<double>(h, const_cast<void*>(buf), U);
        plane_table<double>(h, grad_buf, G);
        e = qds::loss_seed<double>(U, G, geo(h), loss->set, loss->mode, loss->x_begin, loss->x_end, out_dev,
                                   hipStream_t(stream));
    } else {
        qds::cx<float>* U[QDS_NPLANES];
        qds::cx<float>* G[QDS_NPLANES];
        plane_table<float>(h, const_cast<void*>(buf), U);
        plane_table<float>(h, grad_buf, G);
        e = qds::loss_seed<float>(U, G, geo(h), loss->set, loss->mode, loss->x_begin, loss->x_end, out_dev,
                                  hipStream_t(stream));
    }
    if (e != hipSuccess) return fail(h, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    return QDS_OK;
}

qds_status qds_destroy(qds_handle h) {
    if (!h) return QDS_OK;
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    if (h->scratch) (void)hipFree(h->scratch);
    if (h->drive_plane) (void)hipFree(h->drive_plane);
    if (h->psrc) (void)hipFree(h->psrc);
    if (h->pairbuf) (void)hipFree(h->pairbuf);
    if (h->ktab_ev) {
        (void)hipEventSynchronize(h->ktab_ev);
        (void)hipEventDestroy(h->ktab_ev);
    }
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->ev_x) (void)hipEventDestroy(h->ev_x);
    if (h->ev_a) (void)hipEventDestroy(h->ev_a);
    if (h->ktab_dev) (void)hipFree(h->ktab_dev);
    if (h->ktab_pin) (void)hipHostFree(h->ktab_pin);
    delete h;
    return QDS_OK;
}

}  // extern "C"
