// Batched forward over many independent instances (qds_batch_* of
// include/qds.h): per step (or pair of steps), one launch per kernel class
// covering the tiles of every running instance, several steps captured in one
// HIP graph, and an autotuner that picks each class's tile height from timed
// steps of the run.
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "qds_ctx.hpp"

using namespace qdsi;

namespace {

// One kernel launch of a batched step.
struct Launch {
    int slot;     // QDS_TILE_* slot (decides the kernel)
    int M;        // mode count of the class (kernel A and the axion current)
    bool axt;     // kernel A: it advances the axion (instances without the regenerated set)
    int blocks;
    qds::BatchList L;
};

// Launch sequence of one set of running instances, with its device lists and
// the graphs captured for it: key (steps, parity of the buffers at the first
// step).  With pairs, the lists also hold the two-step marches (slots
// QDS_TILE_PAIR0/1), which only pair units launch.
struct Plan {
    std::vector<int> active;
    std::vector<int> tiles;
    bool pairs = false;
    std::vector<int> host;
    void* dev = nullptr;
    std::vector<Launch> launches;
    std::map<std::pair<int, int>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
};

const int kCandA[4] = {8, 16, 24, 32};       // kernel A
const int kCandCur[4] = {4, 6, 8, 16};       // axion current
const int kCandEm[4] = {8, 16, 32, 52};      // the electromagnetic sets alone (kernel B)
const int kCandPair[4] = {16, 32, 52, 86};   // the two-step marches
constexpr int kTunePasses = 2;

}  // namespace

struct qds_batch_ctx {
    std::vector<qds_ctx*> inst;
    int dtype = QDS_F64;
    int tiles[QDS_NTILES];
    int tuned = 0;
    int pairs = 0;                      // this run advances in pairs of steps
    hipStream_t cap = nullptr;          // capture stream (never executes work)
    void* args = nullptr;               // per-run argument tables
    size_t args_cap = 0;
    std::vector<unsigned char> host_args;
    std::vector<Plan*> plans;           // plans and graphs, kept while the tables are unchanged
    // graphs of whole uneven schedules (graph_steps < 0), keyed by the parity
    // of the first step, the tiles and every instance's remaining steps
    std::map<std::vector<int64_t>, std::pair<hipGraph_t, hipGraphExec_t>> whole;
    hipEvent_t done = nullptr;
    bool pending = false;
    // counters since creation: graph launches, graphs instantiated, kernel
    // launches outside graphs, kernel launches inside the launched graphs
    int64_t stats[4] = {0, 0, 0, 0};
    char err[256];
};

namespace {

qds_status bfail(qds_batch_ctx* b, qds_status s, const char* fmt, const char* detail = "") {
    snprintf(b ? b->err : g_err, 256, fmt, detail);
    return s;
}

void release(qds_batch_ctx* b) {
    if (b->pending) {
        (void)hipEventSynchronize(b->done);
        b->pending = false;
    }
    for (Plan* p : b->plans) {
        for (auto& kv : p->graphs) {
            (void)hipGraphExecDestroy(kv.second.second);
            (void)hipGraphDestroy(kv.second.first);
        }
        if (p->dev) (void)hipFree(p->dev);
        delete p;
    }
    b->plans.clear();
    for (auto& kv : b->whole) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    b->whole.clear();
}

int chunks(int nr, int rows) { return (nr + 1 + rows - 1) / rows; }

// Lists of every kernel class for the running instances ``active``.
qds_status build_plan(qds_batch_ctx* b, const std::vector<int>& active, hipStream_t s, Plan** out) {
    Plan* P = new (std::nothrow) Plan();
    if (!P) return bfail(b, QDS_ENOMEM, "out of host memory%s");
    P->active = active;
    P->tiles.assign(b->tiles, b->tiles + QDS_NTILES);
    P->pairs = b->pairs != 0;
    struct Pending { int slot, M; bool axt; std::vector<int> idx, first; };
    std::vector<Pending> pend;
    auto add = [&](int slot, int M, auto pick, auto blocks_of, bool axt = true) {
        Pending q{slot, M, axt, {}, {0}};
        for (int k : active) {
            const qds_ctx* c = b->inst[k];
            if (!pick(c)) continue;
            q.idx.push_back(k);
            q.first.push_back(q.first.back() + blocks_of(c));
        }
        if (!q.idx.empty()) pend.push_back(std::move(q));
    };
    auto has_ax = [](const qds_ctx* c) { return has(c, QDS_P_PHI); };
    auto has_arem = [](const qds_ctx* c) { return has(c, QDS_P_SET1); };
    // kernel A in two launches per mode count: instances with the regenerated
    // set (the axion current advances their axion) and those without
    for (int M = 1; M <= 4; ++M)
        for (int axt = 0; axt < 2; ++axt) {
            const int rows = b->tiles[QDS_TILE_A1 + M - 1];
            add(QDS_TILE_A1 + M - 1, M,
                [&](const qds_ctx* c) { return has_ax(c) && c->M == M && has_arem(c) == !axt; },
                [&](const qds_ctx* c) { return qds::fused_strips(c->g.nx) * chunks(c->g.nr, rows); }, axt != 0);
        }
    {
        const int rows = b->tiles[QDS_TILE_EM0];
        add(QDS_TILE_EM0, 0, [&](const qds_ctx* c) { return !has_ax(c); },
            [&](const qds_ctx* c) { return qds::fused_strips(c->g.nx) * chunks(c->g.nr, rows) * c->M; });
    }
    for (int M = 1; M <= 4; ++M) {
        const int rows = b->tiles[QDS_TILE_CUR1 + M - 1];
        add(QDS_TILE_CUR1 + M - 1, M, [&](const qds_ctx* c) { return has_arem(c) && c->M == M; },
            [&](const qds_ctx* c) { return qds::current_strips(c->g.nx) * chunks(c->g.nr, rows); });
    }
    {
        const int rows = b->tiles[QDS_TILE_EM1];
        add(QDS_TILE_EM1, 0, has_arem,
            [&](const qds_ctx* c) { return qds::fused_strips(c->g.nx) * chunks(c->g.nr, rows) * c->M; });
    }
    if (b->pairs) {
        const int r0 = b->tiles[QDS_TILE_PAIR0], r1 = b->tiles[QDS_TILE_PAIR1];
        add(QDS_TILE_PAIR0, 0, [&](const qds_ctx* c) { return !has_ax(c); },
            [&](const qds_ctx* c) { return qds::pair_strips(c->g.nx) * chunks(c->g.nr, r0) * c->M; });
        add(QDS_TILE_PAIR1, 0, has_arem,
            [&](const qds_ctx* c) { return qds::pair_strips(c->g.nx) * chunks(c->g.nr, r1) * c->M; });
    }
    size_t total = 0;
    for (const Pending& q : pend) {
        if (q.first.back() >= (1 << 30)) {
            delete P;
            return bfail(b, QDS_EUNSUPPORTED, "batched launch exceeds 2^30 workgroups%s");
        }
        total += q.idx.size() + q.first.size();
    }
    P->host.reserve(total);
    std::vector<size_t> off;
    for (const Pending& q : pend) {
        off.push_back(P->host.size());
        P->host.insert(P->host.end(), q.idx.begin(), q.idx.end());
        P->host.insert(P->host.end(), q.first.begin(), q.first.end());
    }
    if (total) {
        if (hipMalloc(&P->dev, total * sizeof(int)) != hipSuccess) {
            delete P;
            return bfail(b, QDS_ENOMEM, "hipMalloc of the batch lists failed%s");
        }
        hipError_t e = hipMemcpyAsync(P->dev, P->host.data(), total * sizeof(int), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            (void)hipFree(P->dev);
            delete P;
            return bfail(b, QDS_EHIP, "list upload failed: %s", hipGetErrorString(e));
        }
    }
    for (size_t q = 0; q < pend.size(); ++q) {
        const int* base = static_cast<const int*>(P->dev) + off[q];
        Launch l;
        l.slot = pend[q].slot;
        l.M = pend[q].M;
        l.axt = pend[q].axt;
        l.blocks = pend[q].first.back();
        l.L.idx = base;
        l.L.first = base + pend[q].idx.size();
        l.L.n = int(pend[q].idx.size());
        l.L.rows = b->tiles[l.slot];
        P->launches.push_back(l);
    }
    b->plans.push_back(P);
    *out = P;
    return QDS_OK;
}

// Argument tables of a run (device, one allocation): fa[2][N] and xa[2][N]
// for single steps from buffer (cur + parity) % 2; with pairs then fp[2][2][N]
// and xp[2][2][N], the pair's first half (into the pair buffer) and second
// half (from it) for each parity.
template <typename T>
const qds::FusedArgs<T>* tab_fa(const qds_batch_ctx* b, int parity) {
    return static_cast<const qds::FusedArgs<T>*>(b->args) + size_t(parity) * b->inst.size();
}
template <typename T>
const qds::AxionArgs<T>* tab_xa(const qds_batch_ctx* b, int parity) {
    const size_t N = b->inst.size();
    return reinterpret_cast<const qds::AxionArgs<T>*>(static_cast<const char*>(b->args) +
                                                      2 * N * sizeof(qds::FusedArgs<T>)) +
           size_t(parity) * N;
}
template <typename T>
const qds::FusedArgs<T>* tab_fp(const qds_batch_ctx* b, int parity, int half) {
    const size_t N = b->inst.size();
    return reinterpret_cast<const qds::FusedArgs<T>*>(static_cast<const char*>(b->args) +
                                                      2 * N * (sizeof(qds::FusedArgs<T>) + sizeof(qds::AxionArgs<T>))) +
           size_t(2 * parity + half) * N;
}
template <typename T>
const qds::AxionArgs<T>* tab_xp(const qds_batch_ctx* b, int parity, int half) {
    const size_t N = b->inst.size();
    return reinterpret_cast<const qds::AxionArgs<T>*>(static_cast<const char*>(b->args) +
                                                      6 * N * sizeof(qds::FusedArgs<T>) +
                                                      2 * N * sizeof(qds::AxionArgs<T>)) +
           size_t(2 * parity + half) * N;
}

// Kernel launches of one single step and of one pair of steps of a plan.
size_t step_launches(const Plan& P) {
    size_t n = 0;
    for (const Launch& l : P.launches) n += l.slot < QDS_TILE_PAIR0;
    return n;
}
size_t pair_launches(const Plan& P) {
    size_t n = 0;
    for (const Launch& l : P.launches) n += l.slot < QDS_TILE_EM0 ? 2 : (l.slot >= QDS_TILE_PAIR0 ? 1 : 0);
    return n;
}

template <typename T>
hipError_t launch_step(const qds_batch_ctx* b, const Plan& P, int parity, hipStream_t s, hipEvent_t* ev) {
    const auto* fa = tab_fa<T>(b, parity);
    const auto* xa = tab_xa<T>(b, parity);
    size_t q = 0;
    for (const Launch& l : P.launches) {
        if (l.slot >= QDS_TILE_PAIR0) continue;
        hipError_t e;
        if (ev && (e = hipEventRecord(ev[2 * q], s)) != hipSuccess) return e;
        if (l.slot < QDS_TILE_CUR1) e = qds::batch_a<T>(fa, l.L, l.M, l.blocks, l.axt, s);
        else if (l.slot < QDS_TILE_EM0) e = qds::batch_current<T>(xa, l.L, l.M, l.blocks, s);
        else e = qds::batch_em<T>(fa, l.L, l.slot == QDS_TILE_EM1 ? 1 : 0, l.blocks, s);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2 * q + 1], s)) != hipSuccess) return e;
        ++q;
    }
    return hipSuccess;
}

// One pair of steps from buffer (cur + parity) % 2: kernel A and the axion
// current of the first step into each instance's pair buffer, those of the
// second step out of it, then the two-step marches (launch order: the kernel-A
// and axion-current classes twice, then the marches; event pairs ev[2q],
// ev[2q + 1] in that order).
template <typename T>
hipError_t launch_pair(const qds_batch_ctx* b, const Plan& P, int parity, hipStream_t s, hipEvent_t* ev) {
    size_t q = 0;
    auto rec = [&](int k) { return ev ? hipEventRecord(ev[2 * q + k], s) : hipSuccess; };
    for (int half = 0; half < 2; ++half) {
        const auto* fp = tab_fp<T>(b, parity, half);
        const auto* xp = tab_xp<T>(b, parity, half);
        for (const Launch& l : P.launches) {
            if (l.slot >= QDS_TILE_EM0) continue;
            hipError_t e;
            if ((e = rec(0)) != hipSuccess) return e;
            e = l.slot < QDS_TILE_CUR1 ? qds::batch_a<T>(fp, l.L, l.M, l.blocks, false, s)
                                       : qds::batch_current<T>(xp, l.L, l.M, l.blocks, s);
            if (e != hipSuccess) return e;
            if ((e = rec(1)) != hipSuccess) return e;
            ++q;
        }
    }
    const auto* fa = tab_fa<T>(b, parity);
    for (const Launch& l : P.launches) {
        if (l.slot < QDS_TILE_PAIR0) continue;
        hipError_t e;
        if ((e = rec(0)) != hipSuccess) return e;
        if ((e = qds::batch_em2<T>(fa, l.L, l.slot == QDS_TILE_PAIR1 ? 1 : 0, true, l.blocks, s)) != hipSuccess) return e;
        if ((e = rec(1)) != hipSuccess) return e;
        ++q;
    }
    return hipSuccess;
}

// The steps of a segment of ``steps`` steps whose first step reads buffer
// parity ``f`` % 2: pairs while two steps remain (with pairs), then single
// steps; returns the buffer flips, adds the kernel launches to *n.
template <typename T>
hipError_t launch_steps(const qds_batch_ctx* b, const Plan& P, int64_t steps, int64_t f, hipStream_t s,
                        int64_t* flips, int64_t* n) {
    int64_t u = 0, k = 0;
    hipError_t e = hipSuccess;
    if (b->pairs)
        for (; u + 2 <= steps && e == hipSuccess; u += 2, ++k) {
            e = launch_pair<T>(b, P, int((f + k) & 1), s, nullptr);
            *n += int64_t(pair_launches(P));
        }
    for (; u < steps && e == hipSuccess; ++u, ++k) {
        e = launch_step<T>(b, P, int((f + k) & 1), s, nullptr);
        *n += int64_t(step_launches(P));
    }
    *flips = k;
    return e;
}

template <typename T>
qds_status run_impl(qds_batch_ctx* b, qds_state* states, const qds_current* J, const qds_axion* ax,
                    const int64_t* n_steps, int graph_steps, int tune, hipStream_t s) {
    const size_t N = b->inst.size();
    // pairs of steps when every instance can take them (the regenerated set
    // on kernel A and the marched axion current, or no axion at all)
    b->pairs = 1;
    for (const qds_ctx* c : b->inst)
        if (!c->pair || (has(c, QDS_P_PHI) && !has(c, QDS_P_SET1))) b->pairs = 0;
    if (b->pairs)
        for (qds_ctx* c : b->inst) {
            if (!has(c, QDS_P_SET1) || c->pairbuf) continue;
            // the instance's pair buffer, as qds_step allocates it
            if (hipMalloc(&c->pairbuf, pairbuf_bytes(c)) != hipSuccess) {
                c->pairbuf = nullptr;
                return bfail(b, QDS_ENOMEM, "hipMalloc of a pair buffer failed%s");
            }
        }
    // argument tables: parity q reads buf[(cur + q) % 2] and writes the other;
    // the step and window counters are not used by the batched kernels (no
    // drive, no window) and are left at zero so that equal states reuse them
    const size_t fbytes = 2 * N * sizeof(qds::FusedArgs<T>);
    const size_t sbytes = fbytes + 2 * N * sizeof(qds::AxionArgs<T>);
    const size_t bytes = sbytes + (b->pairs ? 2 * sbytes : 0);
    std::vector<unsigned char> host(bytes, 0);
    auto* fa = reinterpret_cast<qds::FusedArgs<T>*>(host.data());
    auto* xa = reinterpret_cast<qds::AxionArgs<T>*>(host.data() + fbytes);
    auto* fp = reinterpret_cast<qds::FusedArgs<T>*>(host.data() + sbytes);
    auto* xp = reinterpret_cast<qds::AxionArgs<T>*>(host.data() + sbytes + 2 * fbytes);
    for (size_t k = 0; k < N; ++k) {
        const qds_ctx* c = b->inst[k];
        const qds::StepPlan<T> p0 = make_plan<T>(c, J ? &J[k] : nullptr, ax ? &ax[k] : nullptr);
        qds::StepPlan<T> p2 = p0;   // the second step of a pair: its axion current to the second j_a planes
        for (int q = 0; q < 3; ++q) p2.ja[q] = p0.ja2[q];
        for (int q = 0; q < 2; ++q) {
            void* A = states[k].buf[(states[k].cur + q) & 1];
            void* B = states[k].buf[(states[k].cur + q + 1) & 1];
            qds::FusedArgs<T> f = fused_args<T>(c, p0, A, B);
            qds::AxionArgs<T> x = axion_args<T>(c, p0, A, B);
            memcpy(&fa[q * N + k], &f, sizeof(f));
            memcpy(&xa[q * N + k], &x, sizeof(x));
            if (!b->pairs) continue;
            // instances without the axion only launch the march (from fa)
            void* S = c->pairbuf ? c->pairbuf : B;
            f = fused_args<T>(c, p0, A, S);
            x = axion_args<T>(c, p0, A, S);
            memcpy(&fp[(2 * q) * N + k], &f, sizeof(f));
            memcpy(&xp[(2 * q) * N + k], &x, sizeof(x));
            f = fused_args<T>(c, p2, S, B);
            x = axion_args<T>(c, p2, S, B);
            memcpy(&fp[(2 * q + 1) * N + k], &f, sizeof(f));
            memcpy(&xp[(2 * q + 1) * N + k], &x, sizeof(x));
        }
    }
    hipError_t e;
    if (!(b->args && host == b->host_args)) {
        // the captured graphs and the launch lists hold only the table's device
        // address, so new contents (states whose current buffer flipped, other
        // physics) are uploaded in place once the previous run has finished;
        // only a larger table, which moves, releases them
        if (bytes > b->args_cap) {
            release(b);
        } else if (b->pending) {
            (void)hipEventSynchronize(b->done);
            b->pending = false;
        }
        b->host_args.swap(host);
        if (bytes > b->args_cap) {
            if (b->args) (void)hipFree(b->args);
            b->args = nullptr;
            b->args_cap = 0;
            if (hipMalloc(&b->args, bytes) != hipSuccess)
                return bfail(b, QDS_ENOMEM, "hipMalloc of the batch tables failed%s");
            b->args_cap = bytes;
        }
        e = hipMemcpyAsync(b->args, b->host_args.data(), bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            b->host_args.clear();
            return bfail(b, QDS_EHIP, "table upload failed: %s", hipGetErrorString(e));
        }
    }

    auto running = [&](int64_t t) {
        std::vector<int> a;
        for (size_t k = 0; k < N; ++k)
            if (n_steps[k] > t) a.push_back(int(k));
        return a;
    };
    // t: steps done; f: buffer flips done (a pair flips the buffers once);
    // flips[k]: those of instance k (the parity of its state's buffer index)
    int64_t t = 0, f = 0;
    std::vector<int64_t> flips(N, 0);
    auto advance = [&](const std::vector<int>& act, int64_t steps, int64_t nf) {
        for (int k : act) flips[size_t(k)] += nf;
        t += steps;
        f += nf;
    };
    const int per = b->pairs ? 2 : 1;     // steps per trial of the tuner
    qds_status st;
    auto find_plan = [&](const std::vector<int>& act) -> Plan* {
        for (Plan* p : b->plans)
            if (p->active == act && p->pairs == (b->pairs != 0) &&
                std::equal(p->tiles.begin(), p->tiles.end(), b->tiles))
                return p;
        return nullptr;
    };
    // autotuner: timed trial steps (or pairs) of the run, each candidate tiling twice
    if (tune && !b->tuned) {
        std::vector<int> act = running(0);
        bool enough = !act.empty();
        for (int k : act) enough = enough && n_steps[k] >= 4 * kTunePasses * per;
        if (enough) {
            std::vector<hipEvent_t> evs;
            std::vector<Plan*> trial;
            for (int pass = 0; pass < kTunePasses; ++pass) {
                for (int cand = 0; cand < 4; ++cand) {
                    for (int q = 0; q < 4; ++q) b->tiles[QDS_TILE_A1 + q] = kCandA[cand];
                    for (int q = 0; q < 4; ++q) b->tiles[QDS_TILE_CUR1 + q] = kCandCur[cand];
                    b->tiles[QDS_TILE_EM0] = b->tiles[QDS_TILE_EM1] = kCandEm[cand];
                    b->tiles[QDS_TILE_PAIR0] = b->tiles[QDS_TILE_PAIR1] = kCandPair[cand];
                    Plan* P;
                    if ((st = build_plan(b, act, s, &P)) != QDS_OK) return st;
                    trial.push_back(P);
                    const size_t base = evs.size();
                    const size_t nl = b->pairs ? pair_launches(*P) : step_launches(*P);
                    for (size_t q = 0; q < 2 * nl; ++q) {
                        hipEvent_t ev;
                        if (hipEventCreate(&ev) != hipSuccess) return bfail(b, QDS_EHIP, "event creation failed%s");
                        evs.push_back(ev);
                    }
                    e = b->pairs ? launch_pair<T>(b, *P, int(f & 1), s, evs.data() + base)
                                 : launch_step<T>(b, *P, int(f & 1), s, evs.data() + base);
                    if (e != hipSuccess) return bfail(b, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
                    advance(act, per, 1);
                }
            }
            if (hipStreamSynchronize(s) != hipSuccess) return bfail(b, QDS_EHIP, "tuning run failed%s");
            // per trial, the summed time of the launches of each slot (in the
            // order launch_step or launch_pair issued them)
            float best[QDS_NTILES];
            int pick[QDS_NTILES];
            for (int q = 0; q < QDS_NTILES; ++q) { best[q] = 3.4e38f; pick[q] = -1; }
            size_t ei = 0;
            for (size_t tr = 0; tr < trial.size(); ++tr) {
                const int cand = int(tr % 4);
                float sum[QDS_NTILES];
                bool seen[QDS_NTILES];
                for (int q = 0; q < QDS_NTILES; ++q) { sum[q] = 0.f; seen[q] = false; }
                std::vector<int> order;
                if (b->pairs) {
                    for (int half = 0; half < 2; ++half)
                        for (const Launch& l : trial[tr]->launches)
                            if (l.slot < QDS_TILE_EM0) order.push_back(l.slot);
                    for (const Launch& l : trial[tr]->launches)
                        if (l.slot >= QDS_TILE_PAIR0) order.push_back(l.slot);
                } else {
                    for (const Launch& l : trial[tr]->launches)
                        if (l.slot < QDS_TILE_PAIR0) order.push_back(l.slot);
                }
                for (int slot : order) {
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, evs[ei], evs[ei + 1]) != hipSuccess) {
                        ms = 3.4e38f;
                        (void)hipGetLastError();   // not left for the next launch check
                    }
                    ei += 2;
                    sum[slot] += ms;
                    seen[slot] = true;
                }
                for (int q = 0; q < QDS_NTILES; ++q)
                    if (seen[q] && sum[q] < best[q]) { best[q] = sum[q]; pick[q] = cand; }
            }
            for (int q = 0; q < QDS_NTILES; ++q) {
                const int cand = pick[q] < 0 ? 2 : pick[q];
                b->tiles[q] = q < QDS_TILE_CUR1 ? kCandA[cand]
                                                : (q < QDS_TILE_EM0 ? kCandCur[cand]
                                                                    : (q < QDS_TILE_PAIR0 ? kCandEm[cand] : kCandPair[cand]));
            }
            b->tuned = 1;
            for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
        }
    }
    if (graph_steps < 0) {
        // the whole uneven schedule from step t as one graph: the plan of every
        // segment (running set unchanged) first, its lists uploaded on s, then
        // one capture of all the steps, replayed while the tables, the tiles and
        // the step counts are the same
        std::vector<int64_t> key;
        key.push_back(f & 1);
        key.push_back(b->pairs);
        key.insert(key.end(), b->tiles, b->tiles + QDS_NTILES);
        for (size_t k = 0; k < N; ++k) key.push_back(std::max<int64_t>(n_steps[k] - t, 0));
        std::vector<std::pair<Plan*, int64_t>> segs;
        for (int64_t tt = t;;) {
            std::vector<int> act = running(tt);
            if (act.empty()) break;
            int64_t rem = INT64_MAX;
            for (int k : act) rem = std::min(rem, n_steps[k] - tt);
            Plan* P = find_plan(act);
            if (!P && (st = build_plan(b, act, s, &P)) != QDS_OK) return st;
            segs.emplace_back(P, rem);
            tt += rem;
        }
        if (!segs.empty()) {
            auto it = b->whole.find(key);
            int64_t launches = 0, ff = f;
            hipError_t le = hipSuccess;
            const bool capture = it == b->whole.end();
            hipGraph_t g = nullptr;
            hipGraphExec_t x = nullptr;
            if (capture && (e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed)) != hipSuccess)
                return bfail(b, QDS_EHIP, "capture failed: %s", hipGetErrorString(e));
            for (const auto& sg : segs) {
                // (the launches are only recorded when capturing; the flips and
                // launch counts of a replay are the same)
                int64_t nf = 0;
                if (capture) {
                    if (le == hipSuccess) le = launch_steps<T>(b, *sg.first, sg.second, ff, b->cap, &nf, &launches);
                } else {
                    nf = b->pairs ? sg.second / 2 + sg.second % 2 : sg.second;
                    launches += b->pairs ? (sg.second / 2) * int64_t(pair_launches(*sg.first)) +
                                               (sg.second % 2) * int64_t(step_launches(*sg.first))
                                         : sg.second * int64_t(step_launches(*sg.first));
                }
                for (int k : sg.first->active) flips[size_t(k)] += nf;
                ff += nf;
            }
            if (capture) {
                e = hipStreamEndCapture(b->cap, &g);
                if (le != hipSuccess || e != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return bfail(b, QDS_EHIP, "capture failed: %s", hipGetErrorString(le != hipSuccess ? le : e));
                }
                e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    return bfail(b, QDS_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
                }
                it = b->whole.emplace(key, std::make_pair(g, x)).first;
                b->stats[1] += 1;
            }
            e = hipGraphLaunch(it->second.second, s);
            if (e != hipSuccess) return bfail(b, QDS_EHIP, "graph launch failed: %s", hipGetErrorString(e));
            b->stats[0] += 1;
            b->stats[3] += launches;
        }
    }
    // the run proper, in segments over which the running set is unchanged
    for (; graph_steps >= 0;) {
        std::vector<int> act = running(t);
        if (act.empty()) break;
        int64_t rem = INT64_MAX;
        for (int k : act) rem = std::min(rem, n_steps[k] - t);
        Plan* P = find_plan(act);
        if (!P && (st = build_plan(b, act, s, &P)) != QDS_OK) return st;
        if (graph_steps <= 0) {
            int64_t nf = 0, nl = 0;
            e = launch_steps<T>(b, *P, rem, f, s, &nf, &nl);
            if (e != hipSuccess) return bfail(b, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
            b->stats[2] += nl;
            advance(act, rem, nf);
            continue;
        }
        while (rem > 0) {
            const int seg = int(std::min<int64_t>(rem, graph_steps));
            const std::pair<int, int> key(seg, int(f & 1));
            auto it = P->graphs.find(key);
            int64_t nf = 0, nl = 0;
            if (it == P->graphs.end()) {
                hipGraph_t g = nullptr;
                hipGraphExec_t x = nullptr;
                e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
                if (e != hipSuccess) return bfail(b, QDS_EHIP, "capture failed: %s", hipGetErrorString(e));
                const hipError_t le = launch_steps<T>(b, *P, seg, f, b->cap, &nf, &nl);
                e = hipStreamEndCapture(b->cap, &g);
                if (le != hipSuccess || e != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return bfail(b, QDS_EHIP, "capture failed: %s", hipGetErrorString(le != hipSuccess ? le : e));
                }
                e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    return bfail(b, QDS_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
                }
                it = P->graphs.emplace(key, std::make_pair(g, x)).first;
                b->stats[1] += 1;
            } else {
                nf = b->pairs ? seg / 2 + seg % 2 : seg;
                nl = b->pairs ? int64_t(seg / 2) * int64_t(pair_launches(*P)) + int64_t(seg % 2) * int64_t(step_launches(*P))
                              : int64_t(seg) * int64_t(step_launches(*P));
            }
            e = hipGraphLaunch(it->second.second, s);
            if (e != hipSuccess) return bfail(b, QDS_EHIP, "graph launch failed: %s", hipGetErrorString(e));
            b->stats[0] += 1;
            b->stats[3] += nl;
            advance(act, seg, nf);
            rem -= seg;
        }
    }
    for (size_t k = 0; k < N; ++k) {
        states[k].cur ^= int(flips[k] & 1);
        states[k].step += n_steps[k];
    }
    if (hipEventRecord(b->done, s) != hipSuccess) return bfail(b, QDS_EHIP, "event record failed%s");
    b->pending = true;
    return QDS_OK;
}

}  // namespace

extern "C" {

qds_status qds_batch_create(const qds_handle* handles, int32_t count, qds_batch* out) {
    if (!handles || !out) return bfail(nullptr, QDS_EINVAL, "null argument%s");
    *out = nullptr;
    if (count < 1 || count > 4096) return bfail(nullptr, QDS_EINVAL, "count must be 1..4096%s");
    std::vector<qds_ctx*> v(handles, handles + count);
    for (qds_ctx* c : v) {
        if (!c) return bfail(nullptr, QDS_EINVAL, "null handle%s");
        if (c->g.dtype != v[0]->g.dtype) return bfail(nullptr, QDS_EINVAL, "all instances need one dtype%s");
        if (!fused_ok(c) || c->g.x_bc == QDS_X_WINDOW)
            return bfail(nullptr, QDS_EUNSUPPORTED, "batched instances need <= 4 modes and no moving window%s");
    }
    std::vector<qds_ctx*> sorted = v;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return bfail(nullptr, QDS_EINVAL, "a handle appears twice (its scratch planes would be shared)%s");
    qds_batch_ctx* b = new (std::nothrow) qds_batch_ctx();
    if (!b) return bfail(nullptr, QDS_ENOMEM, "out of host memory%s");
    b->inst = v;
    b->dtype = v[0]->g.dtype;
    for (int q = 0; q < 4; ++q) b->tiles[QDS_TILE_A1 + q] = 16;
    for (int q = 0; q < 4; ++q) b->tiles[QDS_TILE_CUR1 + q] = 16;
    b->tiles[QDS_TILE_EM0] = b->tiles[QDS_TILE_EM1] = 16;
    b->tiles[QDS_TILE_PAIR0] = b->tiles[QDS_TILE_PAIR1] = 32;
    b->err[0] = 0;
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        if (b->cap) (void)hipStreamDestroy(b->cap);
        delete b;
        return bfail(nullptr, QDS_EHIP, "stream or event creation failed%s");
    }
    *out = b;
    return QDS_OK;
}

qds_status qds_batch_run(qds_batch b, qds_state* states, const qds_current* J, const qds_axion* axion,
                         const int64_t* n_steps, int32_t graph_steps, int32_t tune, void* stream) {
    if (!b) return bfail(nullptr, QDS_EINVAL, "null batch%s");
    if (!states || !n_steps) return bfail(b, QDS_EINVAL, "null states or step counts%s");
    if (graph_steps < -1 || graph_steps > 100000) return bfail(b, QDS_EINVAL, "graph_steps must be -1..100000%s");
    for (size_t k = 0; k < b->inst.size(); ++k) {
        qds_ctx* c = b->inst[k];
        if (check_state(c, &states[k]) != QDS_OK) return bfail(b, QDS_ESTATE, "instance state: %s", c->err);
        if (n_steps[k] < 0) return bfail(b, QDS_EINVAL, "negative step count%s");
        if (states[k].step + n_steps[k] >= (int64_t(1) << 31)) return bfail(b, QDS_ESTATE, "step counter would overflow%s");
        if (J && J[k].kind != QDS_J_NONE)
            return bfail(b, QDS_EUNSUPPORTED, "batched instances take no prescribed drive (kind must be NONE)%s");
        if (J && J[k].wp2 != 0.0 && !has(c, QDS_P_JX))
            return bfail(b, QDS_EINVAL, "plasma response needs the plasma planes%s");
        if (!axion && has(c, QDS_P_PHI)) return bfail(b, QDS_EINVAL, "axion parameters missing%s");
    }
    if (b->dtype == QDS_F64)
        return run_impl<double>(b, states, J, axion, n_steps, graph_steps, tune, hipStream_t(stream));
    return run_impl<float>(b, states, J, axion, n_steps, graph_steps, tune, hipStream_t(stream));
}

qds_status qds_batch_get_tiles(qds_batch b, int32_t* tiles, int32_t* tuned) {
    if (!b || !tiles) return bfail(b, QDS_EINVAL, "null argument%s");
    for (int q = 0; q < QDS_NTILES; ++q) tiles[q] = b->tiles[q];
    if (tuned) *tuned = b->tuned;
    return QDS_OK;
}

qds_status qds_batch_set_tiles(qds_batch b, const int32_t* tiles) {
    if (!b || !tiles) return bfail(b, QDS_EINVAL, "null argument%s");
    for (int q = 0; q < QDS_NTILES; ++q)
        if (tiles[q] < 1 || tiles[q] > 1024) return bfail(b, QDS_EINVAL, "tile heights must be 1..1024%s");
    for (int q = 0; q < QDS_NTILES; ++q) b->tiles[q] = tiles[q];
    b->tuned = 1;
    return QDS_OK;
}

qds_status qds_batch_stats(qds_batch b, int64_t* stats) {
    if (!b || !stats) return bfail(b, QDS_EINVAL, "null argument%s");
    for (int q = 0; q < 4; ++q) stats[q] = b->stats[q];
    return QDS_OK;
}

const char* qds_batch_last_error(qds_batch b) { return b ? b->err : g_err; }

qds_status qds_batch_destroy(qds_batch b) {
    if (!b) return QDS_OK;
    release(b);
    if (b->args) (void)hipFree(b->args);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return QDS_OK;
}

}  // extern "C"
