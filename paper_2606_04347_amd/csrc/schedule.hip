// Step schedules of a plan: eager launches, or two steps of every instance
// captured into a HIP graph whose instances run on concurrent branches; and
// the schedule autotuner with its JSON cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "plan.h"

using namespace etd;

namespace {

etd_status eager_steps(etd_plan* plan, int nsteps) {
    for (int k = 0; k < nsteps; ++k)
        for (Instance& I : plan->inst) {
            etd_status st = step_instance(plan, I, plan->stream);
            if (st != ETD_OK) return st;
            ++I.step;
        }
    return ETD_OK;
}

bool rebuilds(const Instance& I, long step) {
    return I.d.model == ETD_COUPLED && I.d.band_threshold > 0.0 && step % I.d.band_rebuild_every == 0;
}

// Double-buffered field pointers of every instance (the coupled step swaps
// phi every step and u in ETD1; two steps restore them).
std::string pointer_state(const etd_plan* plan) {
    std::string k;
    char buf[64];
    for (const Instance& I : plan->inst) {
        snprintf(buf, sizeof buf, "%p,%p;", I.phiA, I.u);
        k += buf;
    }
    return k;
}

// Graph key: pointer state and band-rebuild pattern of the next two steps.
std::string graph_key(const etd_plan* plan) {
    std::string k = pointer_state(plan) + "|";
    for (const Instance& I : plan->inst) {
        k += rebuilds(I, I.step) ? '1' : '0';
        k += rebuilds(I, I.step + 1) ? '1' : '0';
    }
    return k;
}

etd_status ensure_branches(etd_plan* plan, int nb) {
    ScheduleState& S = plan->sched;
    if (!S.fork) HIPCHK(plan, hipEventCreateWithFlags(&S.fork, hipEventDisableTiming));
    if (!S.cap) HIPCHK(plan, hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));   // default priority
    while ((int)S.side.size() < nb) {
        hipStream_t st = nullptr;
        HIPCHK(plan, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));   // default priority
        S.side.push_back(st);
        hipEvent_t e = nullptr;
        HIPCHK(plan, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        S.join.push_back(e);
    }
    return ETD_OK;
}

// Capture two steps of every instance on a private stream (the plan's stream
// may be the null stream, which cannot be captured): fork nb branches, give
// instance i to branch i % nb, join the branches back.  The graph is then
// launched on the plan's stream.  The host-side state (buffer swaps, step
// counters) advances by two steps, as a replay of the graph does on the
// device.
etd_status capture_two_steps(etd_plan* plan, hipGraphExec_t* out) {
    ScheduleState& S = plan->sched;
    const int nb = std::max(1, std::min(S.branches, (int)plan->inst.size()));
    etd_status st = ensure_branches(plan, nb);
    if (st != ETD_OK) return st;
    hipStream_t s = S.cap;
    HIPCHK(plan, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    etd_status bad = ETD_OK;
    hipError_t e = hipEventRecord(S.fork, s);
    for (int b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(S.side[b], S.fork, 0);
    for (int k = 0; k < 2 && e == hipSuccess && bad == ETD_OK; ++k)
        for (size_t i = 0; i < plan->inst.size() && bad == ETD_OK; ++i) {
            Instance& I = plan->inst[i];
            bad = step_instance(plan, I, S.side[i % nb]);
            ++I.step;
        }
    for (int b = 0; b < nb && e == hipSuccess; ++b) {
        e = hipEventRecord(S.join[b], S.side[b]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, S.join[b], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &graph);
    if (bad == ETD_OK && e != hipSuccess)
        bad = fail(&plan->err, ETD_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    if (bad == ETD_OK && ee != hipSuccess)
        bad = fail(&plan->err, ETD_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    if (bad == ETD_OK) {
        const hipError_t ei = hipGraphInstantiateWithFlags(out, graph, 0);
        if (ei != hipSuccess)
            bad = fail(&plan->err, ETD_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (bad == ETD_OK)
        log_msg(2, "plan %p: captured two steps of %zu instance(s) on %d branch(es)", (void*)plan, plan->inst.size(),
                nb);
    return bad;
}

// ------------------------------------------------------------------ autotuner cache
std::string instance_signature(const etd_plan* plan) {
    std::map<std::string, int> count;
    for (const Instance& I : plan->inst) {
        char buf[128];
        snprintf(buf, sizeof buf, "%c%d%c:%dx%dx%d", I.d.model == ETD_COUPLED ? 'c' : 'f', (int)I.d.scheme,
                 I.f32 ? 's' : 'd', I.g.nx, I.g.ny, I.g.nz);
        ++count[buf];
    }
    std::string k;
    for (const auto& kv : count) {
        if (!k.empty()) k += ",";
        k += kv.first + "*" + std::to_string(kv.second);
    }
    return k;
}

bool cache_lookup(const std::string& path, const std::string& key, etd_schedule* out) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    const std::string tag = "\"" + key + "\": {";
    const size_t p = txt.find(tag);
    if (p == std::string::npos) return false;
    int mode = -1, branches = -1, xlines = 0;
    const int got = sscanf(txt.c_str() + p + tag.size(), " \"mode\": %d, \"branches\": %d, \"xlines\": %d", &mode,
                           &branches, &xlines);
    if (got < 2) return false;   // entries without the tile field keep the default tile
    if ((mode != ETD_EXEC_EAGER && mode != ETD_EXEC_GRAPH) || branches < 1 || branches > 64) return false;
    if (xlines != 0 && xlines != 8 && xlines != 16) return false;
    out->mode = mode;
    out->branches = branches;
    out->xlines = xlines;
    return true;
}

void cache_store(const std::string& path, const std::string& key, const etd_schedule& s) {
    std::string txt;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            txt = ss.str();
        }
    }
    char entry[96];
    snprintf(entry, sizeof entry, "{\"mode\": %d, \"branches\": %d, \"xlines\": %d}", s.mode, s.branches,
             s.xlines);
    const std::string line = "\"" + key + "\": " + entry;
    const size_t close = txt.rfind('}');
    if (close == std::string::npos || txt.find(':') == std::string::npos) {
        txt = "{\n" + line + "\n}\n";
    } else {
        size_t end = close;
        while (end > 0 && (txt[end - 1] == '\n' || txt[end - 1] == ' ')) --end;
        txt = txt.substr(0, end) + ",\n" + line + "\n}\n";
    }
    std::ofstream f(path, std::ios::trunc);
    f << txt;
}

// Device state a step carries over to the next one (the double-buffered
// pointers are recorded too, so their parity is restored as well).
struct Snapshot {
    void* base = nullptr;
    std::vector<std::pair<void*, size_t>> parts;   // (device buffer, bytes), copied in order into base
    void *phiA = nullptr, *phiB = nullptr, *u = nullptr, *ut = nullptr;
    long step = 0;
    double A0 = 0.0;
};

}  // namespace

std::vector<std::pair<void*, size_t>> etd::carried_state(const Instance& I) {
    const size_t n = (size_t)I.g.nreal();
    const size_t es = I.d.model == ETD_COUPLED ? (I.f32 ? sizeof(float) : sizeof(double)) : sizeof(double);
    std::vector<std::pair<void*, size_t>> parts;
    parts.push_back({I.scal, sizeof(double) * S_COUNT});
    if (I.d.model == ETD_COUPLED) {
        for (void* p : {I.phiA, I.u, I.lap, I.gx, I.gy, I.gz})
            if (p) parts.push_back({p, n * es});   // gy, gz exist on two-dimensional grids only
        parts.push_back({I.Sphi, 2 * es * (size_t)I.g.nspec()});
        if (I.mask) parts.push_back({I.mask, n});
        // the band list in use until the next rebuild
        if (I.band_idx) parts.push_back({I.band_idx, n * sizeof(int32_t)});
        if (I.band_cnt) parts.push_back({I.band_cnt, (size_t)(band_blocks((long)n) + 2) * sizeof(int64_t)});
        if (I.band_total) parts.push_back({I.band_total, sizeof(int64_t)});
    } else {
        parts.push_back({I.U, n * sizeof(double)});
    }
    if (I.surf) parts.push_back({I.sw.x, n * sizeof(double)});   // the start of the next band solve
    return parts;
}

namespace {

etd_status take_snapshot(etd_plan* plan, Instance& I, Snapshot& v) {
    v.parts = carried_state(I);
    if (I.ring) {   // the trial steps push ring entries too
        v.parts.push_back({I.ring, (size_t)I.ring_cap * kDiagRingFields * sizeof(double)});
        v.parts.push_back({I.ring_meta, 2 * sizeof(int64_t)});
    }
    size_t total = 0;
    for (const auto& pr : v.parts) total += (pr.second + 255) & ~(size_t)255;
    if (hipMalloc(&v.base, total) != hipSuccess) {
        v.base = nullptr;
        return fail(&plan->err, ETD_E_NOMEM, "autotune: no memory for the state snapshot");
    }
    char* dst = (char*)v.base;
    for (const auto& pr : v.parts) {
        HIPCHK(plan, hipMemcpyAsync(dst, pr.first, pr.second, hipMemcpyDeviceToDevice, plan->stream));
        dst += (pr.second + 255) & ~(size_t)255;
    }
    v.phiA = I.phiA;
    v.phiB = I.phiB;
    v.u = I.u;
    v.ut = I.ut;
    v.step = I.step;
    v.A0 = I.A0;
    return ETD_OK;
}

etd_status restore_snapshot(etd_plan* plan, Instance& I, const Snapshot& v) {
    I.phiA = v.phiA;
    I.phiB = v.phiB;
    I.u = v.u;
    I.ut = v.ut;
    I.step = v.step;
    I.A0 = v.A0;
    const char* src = (const char*)v.base;
    for (const auto& pr : v.parts) {
        HIPCHK(plan, hipMemcpyAsync(pr.first, src, pr.second, hipMemcpyDeviceToDevice, plan->stream));
        src += (pr.second + 255) & ~(size_t)255;
    }
    return ETD_OK;
}

}  // namespace

void etd::drop_graphs(etd_plan* plan) {
    for (auto& kv : plan->sched.graphs) (void)hipGraphExecDestroy(kv.second);
    plan->sched.graphs.clear();
}

void etd::release_schedule(etd_plan* plan) {
    drop_graphs(plan);
    ScheduleState& S = plan->sched;
    for (hipStream_t st : S.side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : S.join) (void)hipEventDestroy(e);
    if (S.fork) (void)hipEventDestroy(S.fork);
    if (S.cap) (void)hipStreamDestroy(S.cap);
    S.side.clear();
    S.join.clear();
    S.fork = nullptr;
    S.cap = nullptr;
}

etd_status etd::run_steps(etd_plan* plan, int nsteps) {
    ScheduleState& S = plan->sched;
    bool host_checks = false;   // the band solve reads its convergence flag on the host
    for (const Instance& I : plan->inst) host_checks |= (I.d.flags & ETD_F_SURFACE_NONLOCAL) != 0;
    if (S.mode != ETD_EXEC_GRAPH || plan->timing || host_checks) return eager_steps(plan, nsteps);
    int k = 0;
    for (; k + 2 <= nsteps; k += 2) {
        const std::string key = graph_key(plan);
        auto it = S.graphs.find(key);
        if (it == S.graphs.end()) {
            const std::string before = pointer_state(plan);
            hipGraphExec_t ex = nullptr;
            etd_status st = capture_two_steps(plan, &ex);
            if (st != ETD_OK) return st;
            if (pointer_state(plan) != before) {   // the replay would not match the host state
                (void)hipGraphExecDestroy(ex);
                return fail(&plan->err, ETD_E_STATE, "graph schedule: the step state does not repeat after two steps");
            }
            it = S.graphs.emplace(key, ex).first;
        } else {
            for (Instance& I : plan->inst) I.step += 2;
        }
        HIPCHK(plan, hipGraphLaunch(it->second, plan->stream));
    }
    return eager_steps(plan, nsteps - k);
}

extern "C" {

etd_status etd_set_schedule(etd_plan_t plan, const etd_schedule* sched) {
    if (!plan || !sched) return fail(plan ? &plan->err : nullptr, ETD_E_ARG, "null argument");
    if (sched->mode != ETD_EXEC_EAGER && sched->mode != ETD_EXEC_GRAPH)
        return fail(&plan->err, ETD_E_ARG, "schedule mode must be ETD_EXEC_EAGER or ETD_EXEC_GRAPH");
    if (sched->branches < 1 || sched->branches > 64)
        return fail(&plan->err, ETD_E_ARG, "schedule branches must be in 1..64");
    if (sched->xlines != 0 && sched->xlines != 8 && sched->xlines != 16)
        return fail(&plan->err, ETD_E_ARG, "schedule xlines must be 0, 8 or 16");
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    drop_graphs(plan);
    plan->sched.mode = sched->mode;
    plan->sched.branches = sched->branches;
    plan->sched.xlines = sched->xlines == 16 ? 0 : sched->xlines;
    for (Instance& I : plan->inst) I.xlines = plan->sched.xlines;
    return ETD_OK;
}

etd_status etd_get_schedule(etd_plan_t plan, etd_schedule* out) {
    if (!plan || !out) return fail(plan ? &plan->err : nullptr, ETD_E_ARG, "null argument");
    out->mode = plan->sched.mode;
    out->branches = plan->sched.branches;
    out->xlines = plan->sched.xlines;
    return ETD_OK;
}

etd_status etd_autotune(etd_plan_t plan, int trial_steps, const char* cache_path, etd_schedule* chosen,
                        double* ms_out) {
    if (!plan) return fail(nullptr, ETD_E_ARG, "null plan");
    if (trial_steps < 0) return fail(&plan->err, ETD_E_ARG, "trial_steps must be >= 0");
    for (const Instance& I : plan->inst)
        if (!I.has_state) return fail(&plan->err, ETD_E_STATE, "autotune before set_state");
    // the schedules, then the fastest of them with 8-line tiles in the FP32
    // ETD x pass (only where an instance takes that pass)
    etd_schedule cand[ETD_AUTOTUNE_CANDIDATES] = {{ETD_EXEC_EAGER, 1, 0}, {ETD_EXEC_GRAPH, 1, 0},
                                                   {ETD_EXEC_GRAPH, 2, 0},  {ETD_EXEC_GRAPH, 4, 0},
                                                   {ETD_EXEC_GRAPH, 8, 0},  {ETD_EXEC_GRAPH, 16, 0},
                                                   {ETD_EXEC_GRAPH, 32, 0}, {ETD_EXEC_EAGER, 1, 8}};
    bool tile_knob = false;
    for (const Instance& I : plan->inst)
        tile_knob = tile_knob || (I.d.model == ETD_COUPLED && I.f32 && I.g.nx > 1);
    if (ms_out)
        for (int c = 0; c < ETD_AUTOTUNE_CANDIDATES; ++c) ms_out[c] = -1.0;
    hipDeviceProp_t prop;
    HIPCHK(plan, hipGetDeviceProperties(&prop, plan->device));
    const std::string key = std::string(prop.gcnArchName) + "|" + instance_signature(plan);
    etd_schedule best{ETD_EXEC_EAGER, 1};
    // the cache file: the argument, else the environment's ETD_AUTOTUNE_CACHE
    if (!cache_path || !*cache_path) {
        const char* env = std::getenv("ETD_AUTOTUNE_CACHE");
        cache_path = (env && *env) ? env : nullptr;
    }
    if (cache_path && cache_lookup(cache_path, key, &best)) {
        log_msg(2, "autotune %s: cached mode %d, %d branch(es), %d-line x tile (%s)", key.c_str(), best.mode,
                best.branches, best.xlines ? best.xlines : 16, cache_path);
        etd_status st = etd_set_schedule(plan, &best);
        if (st == ETD_OK && chosen) *chosen = best;
        return st;
    }
    const int trial = std::max(2, trial_steps + (trial_steps & 1));
    const int ninst = (int)plan->inst.size();
    hipStream_t s = plan->stream;
    // exact device copies of everything a step carries over, and the host-side state
    std::vector<Snapshot> saved(ninst);
    auto release = [&] {
        for (Snapshot& v : saved)
            if (v.base) (void)hipFree(v.base);
    };
    for (int i = 0; i < ninst; ++i) {
        etd_status st = take_snapshot(plan, plan->inst[i], saved[i]);
        if (st != ETD_OK) {
            release();
            return st;
        }
    }
    const etd_schedule old{plan->sched.mode, plan->sched.branches, plan->sched.xlines};
    double best_ms = -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    etd_status st = ETD_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        st = fail(&plan->err, ETD_E_HIP, "autotune: hipEventCreate failed");
    for (int c = 0; c < ETD_AUTOTUNE_CANDIDATES && st == ETD_OK; ++c) {
        if (cand[c].mode == ETD_EXEC_GRAPH && cand[c].branches > 1 && cand[c].branches > ninst) continue;
        if (cand[c].xlines == 8) {   // the last candidate: the best schedule so far, 8-line tiles
            if (!tile_knob) continue;
            cand[c].mode = best.mode;
            cand[c].branches = best.branches;
        }
        if ((st = etd_set_schedule(plan, &cand[c])) != ETD_OK) break;
        if ((st = run_steps(plan, 2)) != ETD_OK) break;   // warm-up (captures the graph)
        float ms = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess) st = fail(&plan->err, ETD_E_HIP, "autotune: event record");
        if (st == ETD_OK) st = run_steps(plan, trial);
        if (st == ETD_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = fail(&plan->err, ETD_E_HIP, "autotune: event timing");
        if (st != ETD_OK) break;
        const double per = ms / trial;
        log_msg(2, "autotune candidate %d (mode %d, %d branch(es), %d-line x tile): %.4f ms/step", c, cand[c].mode,
                cand[c].branches, cand[c].xlines ? cand[c].xlines : 16, per);
        if (ms_out) ms_out[c] = per;
        if (best_ms < 0.0 || per < best_ms) {
            best_ms = per;
            best = cand[c];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // restore every state and the host-side quantities
    for (int i = 0; i < ninst; ++i) {
        etd_status sr = restore_snapshot(plan, plan->inst[i], saved[i]);
        if (sr != ETD_OK && st == ETD_OK) st = sr;
    }
    if (st == ETD_OK && hipStreamSynchronize(s) != hipSuccess)
        st = fail(&plan->err, ETD_E_HIP, "autotune: restoring the states failed");
    release();
    drop_graphs(plan);   // captured with the trial states' arguments
    if (st != ETD_OK) {
        (void)etd_set_schedule(plan, &old);
        return st;
    }
    st = etd_set_schedule(plan, &best);
    if (st != ETD_OK) return st;
    if (chosen) *chosen = best;
    log_msg(2, "autotune %s: chose mode %d, %d branch(es), %d-line x tile", key.c_str(), best.mode, best.branches,
            best.xlines ? best.xlines : 16);
    if (cache_path) cache_store(cache_path, key, best);
    return ETD_OK;
}

}  // extern "C"
