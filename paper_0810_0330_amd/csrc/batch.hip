// Uneven batches of independent systems, each single-seeded.
//
// The seed phase of every system has static control flow (exactly m steps,
// reorthogonalization at known steps), so all of them are captured into one
// HIP graph: the caller's stream forks into one stream per system, each
// system's Lanczos kernels are enqueued on its own branch, and the branches
// join back.  One graph launch then advances every lattice concurrently: the
// small lattices, which cannot fill the GPU alone, overlap with the large
// ones.  The instantiated graph is cached and replayed when the same argument
// set is solved again: a graph bakes in its pointers, sizes, operator
// parameters (kappa, links, lattice) and stencil launch shapes, so the cache
// key holds all of them and each op's generation number, and destroying an
// op drops the graphs recorded for it.
//
// The rest is data dependent: each system's final seed state is read, x^1
// formed and the other right-hand sides projected on the system's stream.
// Every column is then finished with CG, all systems from one host thread:
// each system's fixed chunk of CG iterations (per-column masks on the device)
// is captured once into a graph (cached like the seed graph) and replayed on
// the system's stream, and between replays the host checks every system
// (stall rules, reliable updates, the final true-residual check).  Before any
// of this, every lattice's stencil shapes (one column for the seed, k columns
// for CG) are tuned one system at a time, so no shape is timed while other
// systems share the chip.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "sc_internal.h"

namespace sc {

namespace {

struct SysPlan {
    size_t v_off, a_off, b_off, seed_off, seed_bytes, proj_off, proj_bytes, cg_off, cg_bytes;
    sc_dtype vdt;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

std::vector<SysPlan> plan_batch(int nsys, const sc_batch_system* sys, size_t* total) {
    std::vector<SysPlan> p(nsys);
    size_t off = 0;
    for (int i = 0; i < nsys; ++i) {
        const sc_op* op = sys[i].op;
        const bool single = sys[i].mixed != 0;
        const bool cpl = is_complex(op->dtype);
        SysPlan& q = p[i];
        q.vdt = single ? single_of(op->dtype) : op->dtype;
        q.v_off = off;
        off = align256(off + (size_t)(sys[i].m + 1) * op->n * dtype_bytes(q.vdt));
        q.a_off = off;
        off = align256(off + (size_t)sys[i].m * 8);
        q.b_off = off;
        off = align256(off + (size_t)(sys[i].m + 1) * 8);
        q.seed_off = off;
        q.seed_bytes = seed_workspace(op, sys[i].m, single);
        off = align256(off + q.seed_bytes);
        q.proj_off = off;
        q.proj_bytes = project_workspace(op->n, sys[i].m, sys[i].k - 1, cpl);
        off = align256(off + q.proj_bytes);
        q.cg_off = off;
        q.cg_bytes = cg_workspace(op, sys[i].k, single);
        off = align256(off + q.cg_bytes);
    }
    *total = off + 256;
    return p;
}

// A cached instantiated graph for one argument set.
struct GraphKey {
    std::vector<char> bytes;
    bool operator==(const GraphKey& o) const { return bytes == o.bytes; }
};
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> gens;  // generations of the ops the graph was recorded for
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // most recent last
constexpr size_t kGraphCache = 32;  // seed graphs and per-system CG chunk graphs

void key_put(GraphKey& k, const void* p, size_t n) {
    const char* c = (const char*)p;
    k.bytes.insert(k.bytes.end(), c, c + n);
}

// what a captured seed phase bakes in of its operator: the op's contents and
// the stencil shape its one-column passes were tuned to
void key_put_op(GraphKey& k, const sc_op* op, bool single) {
    auto put = [&](const void* p, size_t n) { key_put(k, p, n); };
    put(&op, sizeof op);
    put(&op->gen, sizeof op->gen);
    put(&op->kind, sizeof op->kind);
    put(&op->n, sizeof op->n);
    put(&op->dtype, sizeof op->dtype);
    put(&op->nx, sizeof op->nx);
    put(&op->ny, sizeof op->ny);
    put(&op->d, sizeof op->d);
    put(op->dims, sizeof op->dims);
    put(&op->U64, sizeof op->U64);
    put(&op->U32, sizeof op->U32);
    put(&op->kappa, sizeof op->kappa);
    put(&op->antiperiodic, sizeof op->antiperiodic);
    put(&op->su3, sizeof op->su3);
    int variant = -1;
    if (has_links(op)) {
        float us[SC_WILSON_VARIANTS];
        (void)wilson_tune_query(op, single, 1, &variant, us);
    }
    put(&variant, sizeof variant);
}

GraphKey make_key(int nsys, const sc_batch_system* sys, const void* work, hipStream_t s) {
    GraphKey k;
    auto put = [&](const void* p, size_t n) { key_put(k, p, n); };
    put(&nsys, sizeof nsys);
    put(&work, sizeof work);
    put(&s, sizeof s);
    for (int i = 0; i < nsys; ++i) {
        key_put_op(k, sys[i].op, sys[i].mixed != 0);
        put(&sys[i].B_dev, sizeof sys[i].B_dev);
        put(&sys[i].ldb, sizeof sys[i].ldb);
        put(&sys[i].X_dev, sizeof sys[i].X_dev);
        put(&sys[i].ldx, sizeof sys[i].ldx);
        put(&sys[i].k, sizeof sys[i].k);
        put(&sys[i].m, sizeof sys[i].m);
        put(&sys[i].reorth_freq, sizeof sys[i].reorth_freq);
        put(&sys[i].mixed, sizeof sys[i].mixed);
    }
    return k;
}

// The graph of one system's CG chunk: its kGraphChunk iterations captured
// on the system's stream.  The key holds everything the captured launches
// bake in (operator, buffers, workspace, the tuned shape of the k-column
// passes, the state copy the chunk starts from); an even chunk returns the
// CG object to the same state copy, so the graph replays as captured.
constexpr int kGraphChunk = 8;
static_assert(kGraphChunk % 2 == 0, "a chunk must return to its starting state copy");

GraphKey make_cg_key(const sc_batch_system& b, const void* cg_work, int cur) {
    GraphKey k;
    auto put = [&](const void* p, size_t n) {
        const char* c = (const char*)p;
        k.bytes.insert(k.bytes.end(), c, c + n);
    };
    const char tag = 'C';
    put(&tag, 1);
    const sc_op* op = b.op;
    put(&op, sizeof op);
    put(&op->gen, sizeof op->gen);
    put(&op->kind, sizeof op->kind);
    put(&op->n, sizeof op->n);
    put(&op->dtype, sizeof op->dtype);
    put(&op->nx, sizeof op->nx);
    put(&op->ny, sizeof op->ny);
    put(&op->d, sizeof op->d);
    put(op->dims, sizeof op->dims);
    put(&op->U64, sizeof op->U64);
    put(&op->U32, sizeof op->U32);
    put(&op->kappa, sizeof op->kappa);
    put(&op->antiperiodic, sizeof op->antiperiodic);
    put(&op->su3, sizeof op->su3);  // the FP32 passes' link form
    int variant = -1;
    if (has_links(op)) {
        float us[SC_WILSON_VARIANTS];
        (void)wilson_tune_query(op, b.mixed != 0, b.k, &variant, us);
    }
    put(&variant, sizeof variant);
    put(&b.B_dev, sizeof b.B_dev);
    put(&b.ldb, sizeof b.ldb);
    put(&b.X_dev, sizeof b.X_dev);
    put(&b.ldx, sizeof b.ldx);
    put(&b.k, sizeof b.k);
    put(&b.mixed, sizeof b.mixed);
    put(&cg_work, sizeof cg_work);
    put(&cur, sizeof cur);
    return k;
}

// Finds or records the chunk graph of one system (*exec stays null, and the
// chunk runs eagerly, if the stream cannot be captured)
sc_status chunk_graph(const sc_batch_system& b, const void* cg_work, CGRun& cg, hipGraphExec_t* exec) {
    *exec = nullptr;
    GraphKey key = make_cg_key(b, cg_work, cg.state_index());
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (size_t j = 0; j < g_graphs.size(); ++j)
            if (g_graphs[j].key == key) {
                *exec = g_graphs[j].exec;
                GraphEntry e = g_graphs[j];
                g_graphs.erase(g_graphs.begin() + j);
                g_graphs.push_back(e);
                return SC_OK;
            }
    }
    hipStream_t s = cg.stream();
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return SC_OK;
    const int before = cg.state_index();
    const sc_status st = cg.iterate(kGraphChunk);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(s, &graph);
    if (st != SC_OK || ce != hipSuccess || cg.state_index() != before) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st != SC_OK) return st;
        set_error(std::string("batch_solve: chunk capture failed: ") + hipGetErrorString(ce));
        return SC_ERR_HIP;
    }
    hipGraphExec_t e = nullptr;
    const hipError_t ie = hipGraphInstantiate(&e, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        set_error(std::string("batch_solve: chunk graph instantiation failed: ") + hipGetErrorString(ie));
        return SC_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back({key, e, {b.op->gen}});
    *exec = e;
    return SC_OK;
}

}  // namespace

void batch_forget_op(const sc_op* op) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (size_t j = 0; j < g_graphs.size();) {
        const auto& g = g_graphs[j].gens;
        if (std::find(g.begin(), g.end(), op->gen) != g.end()) {
            (void)hipGraphExecDestroy(g_graphs[j].exec);
            g_graphs.erase(g_graphs.begin() + j);
        } else {
            ++j;
        }
    }
}

// One system's seed phase (seed_enqueue_any) replayed on `s` from a cached
// graph, captured on a private stream the first time these arguments come
// (the caller's stream may be the null stream, which cannot capture).  The
// key holds everything the captured launches bake in.  While `s` is itself
// being captured the phase is launched directly into that capture.  The
// operator's stencil shapes must be tuned beforehand (seed_pretune).
sc_status seed_enqueue_cached(const sc_op* op, const void* b1, void* x1, int m, int freq, void* V, int64_t ldv,
                              sc_dtype vdt, double* alpha, double* beta, const SeedWork& w, hipStream_t s,
                              bool single) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SC_HIP(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return seed_enqueue_any(op, b1, x1, m, freq, V, ldv, vdt, alpha, beta, w, s);
    GraphKey key;
    const int tag = -1;  // batch keys start with their system count, >= 1
    key_put(key, &tag, sizeof tag);
    key_put(key, &s, sizeof s);
    key_put_op(key, op, single);
    for (const void* p : {b1, (const void*)x1, (const void*)V, (const void*)alpha, (const void*)beta})
        key_put(key, &p, sizeof p);
    key_put(key, &ldv, sizeof ldv);
    key_put(key, &vdt, sizeof vdt);
    key_put(key, &m, sizeof m);
    key_put(key, &freq, sizeof freq);
    key_put(key, &w, sizeof w);  // the workspace's carved pointers
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (size_t j = 0; j < g_graphs.size(); ++j)
            if (g_graphs[j].key == key) {
                exec = g_graphs[j].exec;
                GraphEntry e = g_graphs[j];
                g_graphs.erase(g_graphs.begin() + j);
                g_graphs.push_back(e);
                break;
            }
    }
    if (!exec) {
        hipStream_t cap = nullptr;
        SC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        sc_status st = SC_OK;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = seed_enqueue_any(op, b1, x1, m, freq, V, ldv, vdt, alpha, beta, w, cap);
            e = hipStreamEndCapture(cap, &graph);
        }
        (void)hipStreamDestroy(cap);
        if (st != SC_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (st != SC_OK) return st;
            set_error(std::string("seed phase capture failed: ") + hipGetErrorString(e));
            return SC_ERR_HIP;
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            set_error(std::string("seed phase graph instantiation failed: ") + hipGetErrorString(e));
            return SC_ERR_HIP;
        }
        std::lock_guard<std::mutex> lk(g_graph_mu);
        if (g_graphs.size() >= kGraphCache) {
            (void)hipGraphExecDestroy(g_graphs.front().exec);
            g_graphs.erase(g_graphs.begin());
        }
        g_graphs.push_back({key, exec, {op->gen}});
    }
    SC_HIP(hipGraphLaunch(exec, s));
    return SC_OK;
}

size_t batch_workspace(int nsys, const sc_batch_system* sys) {
    size_t total = 0;
    plan_batch(nsys, sys, &total);
    return total;
}

sc_status batch_solve(int nsys, sc_batch_system* sys, void* work, size_t work_bytes, hipStream_t s) {
    size_t total = 0;
    std::vector<SysPlan> plan = plan_batch(nsys, sys, &total);
    char* base = (char*)(((uintptr_t)work + 255) & ~uintptr_t(255));
    if ((size_t)(base - (char*)work) + total - 256 > work_bytes) {
        set_error("batch_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    std::vector<SeedWork> sw(nsys);
    for (int i = 0; i < nsys; ++i) {
        bool ok = false;
        sw[i] = seed_carve(base + plan[i].seed_off, plan[i].seed_bytes, sys[i].op, sys[i].m, sys[i].mixed != 0, &ok);
        if (!ok) {
            set_error("batch_solve: seed workspace carving failed");
            return SC_ERR_WORKSPACE;
        }
    }
    // one stream per system, forked from and joined back to a private capture
    // stream (the caller's stream may be the null stream, which cannot capture)
    std::vector<hipStream_t> ss(nsys + 1, nullptr);
    std::vector<hipEvent_t> ev(nsys + 1, nullptr);
    auto cleanup = [&]() {
        for (auto& x : ss)
            if (x) (void)hipStreamDestroy(x);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (int i = 0; i <= nsys; ++i)
        if (hipStreamCreateWithFlags(&ss[i], hipStreamNonBlocking) != hipSuccess) {
            cleanup();
            set_error("batch_solve: stream creation failed");
            return SC_ERR_HIP;
        }
    for (auto& e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            cleanup();
            set_error("batch_solve: event creation failed");
            return SC_ERR_HIP;
        }

    sc_status st = SC_OK;
    // tune each lattice's stencil shapes before any capture and before the
    // systems run concurrently (a shape timed while other systems' kernels
    // share the chip would be chosen on contended timings): the seed phase's
    // one-column passes and the CG passes over the system's k columns
    for (int i = 0; i < nsys && st == SC_OK; ++i) {
        st = seed_pretune(sys[i].op, sys[i].mixed != 0, sw[i], s);
        if (st == SC_OK && sys[i].k > 1)
            st = cg_pretune(sys[i].op, sys[i].mixed, sys[i].k, base + plan[i].cg_off, plan[i].cg_bytes, s);
    }
    if (st != SC_OK) {
        cleanup();
        return st;
    }

    // ---- seed phases: one graph over all systems
    GraphKey key = make_key(nsys, sys, work, s);
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (size_t j = 0; j < g_graphs.size(); ++j)
            if (g_graphs[j].key == key) {
                exec = g_graphs[j].exec;
                GraphEntry e = g_graphs[j];
                g_graphs.erase(g_graphs.begin() + j);
                g_graphs.push_back(e);
                break;
            }
    }
    if (!exec) {
        hipGraph_t graph = nullptr;
        hipStream_t cap = ss[nsys];
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            cleanup();
            set_error("batch_solve: stream capture could not start");
            return SC_ERR_HIP;
        }
        // a failed record or wait ends the capture with an error (checked below)
        bool evfail = hipEventRecord(ev[nsys], cap) != hipSuccess;
        for (int i = 0; i < nsys && st == SC_OK && !evfail; ++i) {
            const sc_batch_system& b = sys[i];
            if (hipStreamWaitEvent(ss[i], ev[nsys], 0) != hipSuccess) {
                evfail = true;
                break;
            }
            const int64_t N2 = b.op->n * (is_complex(b.op->dtype) ? 2 : 1);
            // X = 0: the seed refines column 0 in place (x0 = 0)
            st = fill<double>((double*)b.X_dev, (b.k - 1) * b.ldx * (is_complex(b.op->dtype) ? 2 : 1) + N2, 0.0,
                              ss[i]);
            if (st == SC_OK)
                st = seed_enqueue_any(b.op, b.B_dev, b.X_dev, b.m, b.reorth_freq, base + plan[i].v_off, b.op->n,
                                      plan[i].vdt, (double*)(base + plan[i].a_off), (double*)(base + plan[i].b_off),
                                      sw[i], ss[i]);
            if (hipEventRecord(ev[i], ss[i]) != hipSuccess || hipStreamWaitEvent(cap, ev[i], 0) != hipSuccess)
                evfail = true;
        }
        const hipError_t ce = hipStreamEndCapture(cap, &graph);
        if (st != SC_OK || evfail || ce != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            cleanup();
            if (st == SC_OK && evfail) {
                set_error("batch_solve: event record or wait failed during capture");
                st = SC_ERR_HIP;
            } else if (st == SC_OK) {
                set_error(std::string("batch_solve: capture failed: ") + hipGetErrorString(ce));
                st = SC_ERR_HIP;
            }
            return st;
        }
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            cleanup();
            set_error(std::string("batch_solve: graph instantiation failed: ") + hipGetErrorString(ie));
            return SC_ERR_HIP;
        }
        std::lock_guard<std::mutex> lk(g_graph_mu);
        if (g_graphs.size() >= kGraphCache) {
            (void)hipGraphExecDestroy(g_graphs.front().exec);
            g_graphs.erase(g_graphs.begin());
        }
        std::vector<uint64_t> gens;
        for (int i = 0; i < nsys; ++i) gens.push_back(sys[i].op->gen);
        g_graphs.push_back({key, exec, gens});
    }
    if (hipGraphLaunch(exec, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        set_error("batch_solve: graph launch failed");
        return SC_ERR_HIP;
    }

    // ---- per system: x^1 and the projection, enqueued on the system's stream
    std::vector<sc_status> res(nsys, SC_OK), seed_st(nsys, SC_OK);
    std::vector<std::string> err(nsys);
    auto fail = [&](int i, sc_status r) {
        res[i] = r;
        if (r < 0) err[i] = sc_last_error();
    };
    for (int i = 0; i < nsys; ++i) {
        sc_batch_system& b = sys[i];
        const SysPlan& q = plan[i];
        sc_status r = seed_finalize_any(b.op, b.X_dev, base + q.v_off, b.op->n, q.vdt, (double*)(base + q.a_off),
                                        (double*)(base + q.b_off), &b.m_done, sw[i], ss[i], &seed_st[i]);
        if (r == SC_OK && (seed_st[i] == SC_ERR_NOT_PD || seed_st[i] == SC_ERR_NONFINITE)) r = seed_st[i];
        const size_t eb = dtype_bytes(b.op->dtype);
        if (r == SC_OK && b.k > 1 && b.m_done >= 1)
            r = project_impl(b.op->n, base + q.v_off, b.op->n, q.vdt, b.m_done, (double*)(base + q.a_off),
                             (double*)(base + q.b_off), b.op->dtype, (const char*)b.B_dev + b.ldb * eb, b.ldb, b.k - 1,
                             (char*)b.X_dev + b.ldx * eb, b.ldx, base + q.proj_off, q.proj_bytes, ss[i]);
        fail(i, r);
    }

    // ---- CG of every system, advanced together from one host thread: each
    // system's fixed chunk of kGraphChunk iterations (column masks on the
    // device) is captured once into a graph, cached like the seed graph, and
    // replayed on the system's stream; the host then checks every system
    // (stall rules, reliable updates) and replays again
    std::vector<std::unique_ptr<CGRun>> cg(nsys);
    std::vector<hipGraphExec_t> chunk(nsys, nullptr);
    std::vector<bool> done(nsys, true);
    for (int i = 0; i < nsys; ++i) {
        if (res[i] != SC_OK) continue;
        sc_batch_system& b = sys[i];
        sc_status r = SC_OK;
        cg[i] = cg_make(b.op, b.mixed, b.B_dev, b.ldb, b.X_dev, b.ldx, b.k, b.tol, b.maxit, base + plan[i].cg_off,
                        plan[i].cg_bytes, ss[i], &r);
        if (cg[i]) r = cg[i]->start();
        if (r == SC_OK) r = chunk_graph(sys[i], base + plan[i].cg_off, *cg[i], &chunk[i]);
        if (r != SC_OK) {
            fail(i, r);
            cg[i].reset();
            continue;
        }
        done[i] = false;
    }
    for (;;) {
        bool left = false;
        for (int i = 0; i < nsys; ++i)
            if (!done[i] && cg[i]->any_active()) {
                const sc_status r = chunk[i] ? (hipGraphLaunch(chunk[i], ss[i]) == hipSuccess ? SC_OK : SC_ERR_HIP)
                                             : cg[i]->iterate(kGraphChunk);
                if (r != SC_OK) {
                    if (r == SC_ERR_HIP) set_error("batch_solve: chunk graph launch failed");
                    fail(i, r);
                    done[i] = true;
                }
            }
        for (int i = 0; i < nsys; ++i) {
            if (done[i]) continue;
            sc_status r = SC_OK;
            if (cg[i]->any_active()) {
                bool any = false;
                r = cg[i]->check(&any);
            } else {
                bool again = false;
                r = cg[i]->verify(&again);
                if (r == SC_OK && !again) {
                    sc_batch_system& b = sys[i];
                    cg[i]->results(b.iters, b.relres, &r);
                    if (r == SC_OK && seed_st[i] == SC_BREAKDOWN) r = SC_BREAKDOWN;
                    done[i] = true;
                }
            }
            if (r < 0) {
                fail(i, r);
                done[i] = true;
            } else if (done[i]) {
                res[i] = r;
            }
            left |= !done[i];
        }
        if (!left) break;
    }
    for (int i = 0; i < nsys; ++i) sys[i].status = res[i];
    // join: the caller's stream waits for every system's stream
    bool joined = true;
    for (int i = 0; i < nsys; ++i)
        joined = joined && hipEventRecord(ev[i], ss[i]) == hipSuccess && hipStreamWaitEvent(s, ev[i], 0) == hipSuccess;
    joined = joined && hipStreamSynchronize(s) == hipSuccess;
    if (!joined) {
        for (auto& x : ss) (void)hipStreamSynchronize(x);
        cleanup();
        set_error("batch_solve: joining the per-system streams failed");
        return SC_ERR_HIP;
    }
    cleanup();
    sc_status out = SC_OK;
    for (int i = 0; i < nsys; ++i) {
        if (res[i] < 0) {
            set_error("batch_solve: system " + std::to_string(i) + ": " + err[i]);
            return res[i];
        }
        if (res[i] == SC_NOT_CONVERGED) out = SC_NOT_CONVERGED;
        else if (res[i] == SC_BREAKDOWN && out == SC_OK) out = SC_BREAKDOWN;
    }
    return out;
}

}  // namespace sc
