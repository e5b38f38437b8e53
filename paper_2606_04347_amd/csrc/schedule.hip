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

#include "launch.h"
#include "plan.h"

using namespace etd;

thread_local LaunchRecorder* etd::g_launch_recorder = nullptr;

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

// Grouped schedule.  Two steps of every instance are recorded (launch_k
// records instead of launching; the recording stream is under capture, so
// any other device work a step would enqueue shows up as a graph node and is
// refused), the instances whose launch sequences agree (kernel, grid, block,
// LDS, argument size: one shape and configuration) form a group, and each
// recorded pass of a group becomes ONE launch of the grouped twin over
// gridDim.x tiles by as many rows as the group has instances, reading its
// arguments from a device table.  The groups are spread round-robin over
// min(branches, groups) concurrent branches of one captured graph.
// Instances the grouped passes cover: coupled, three-dimensional, without a
// band, diagnostics ring, mass projection or band solve.
bool groupable(const Instance& I) {
    return I.d.model == ETD_COUPLED && I.g.nx > 1 && !(I.d.band_threshold > 0.0) && !I.ring &&
           !(I.d.flags & (ETD_F_MASS_PROJECT | ETD_F_SURFACE_NONLOCAL));
}

// The host-side state a step advances (restored when a capture fails).
struct HostStepState {
    void *phiA, *phiB, *u, *ut;
    long step;
};

etd_status record_two_steps(etd_plan* plan, std::vector<LaunchRecorder>& rec) {
    ScheduleState& S = plan->sched;
    if (!S.rec) HIPCHK(plan, hipStreamCreateWithFlags(&S.rec, hipStreamNonBlocking));   // default priority
    rec.assign(plan->inst.size(), LaunchRecorder{});
    for (int k = 0; k < 2; ++k)
        for (size_t i = 0; i < plan->inst.size(); ++i) {
            Instance& I = plan->inst[i];
            HIPCHK(plan, hipStreamBeginCapture(S.rec, hipStreamCaptureModeRelaxed));
            g_launch_recorder = &rec[i];
            const etd_status st = step_instance(plan, I, S.rec);
            g_launch_recorder = nullptr;
            ++I.step;
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(S.rec, &gr);
            size_t nodes = 0;
            if (e == hipSuccess && gr) e = hipGraphGetNodes(gr, nullptr, &nodes);
            if (gr) (void)hipGraphDestroy(gr);
            if (st != ETD_OK) return st;
            if (e != hipSuccess)
                return fail(&plan->err, ETD_E_HIP, std::string("grouped schedule: recording: ") + hipGetErrorString(e));
            if (nodes)
                return fail(&plan->err, ETD_E_ARG,
                            "grouped schedule: instance " + std::to_string(i) +
                                " enqueues work the grouped passes do not cover (band list, diagnostics ring, mass "
                                "projection, band solve, two-dimensional grid or fixed model); use ETD_EXEC_GRAPH");
        }
    return ETD_OK;
}

std::string launch_signature(const LaunchRecorder& r) {
    std::string k;
    char buf[128];
    for (const LaunchRecord& op : r.ops) {
        snprintf(buf, sizeof buf, "%p:%u.%u.%u:%u:%zu:%zu;", op.fn, op.grid.x, op.grid.y, op.grid.z, op.block.x, op.smem,
                 op.args.size());
        k += buf;
    }
    return k;
}

etd_status capture_grouped_steps(etd_plan* plan, ScheduleState::Captured* out);

// On failure nothing ran and the host-side state is as before.
etd_status capture_grouped(etd_plan* plan, ScheduleState::Captured* out) {
    std::vector<HostStepState> before;
    for (const Instance& I : plan->inst) before.push_back({I.phiA, I.phiB, I.u, I.ut, I.step});
    const etd_status st = capture_grouped_steps(plan, out);
    if (st != ETD_OK)
        for (size_t i = 0; i < plan->inst.size(); ++i) {
            Instance& I = plan->inst[i];
            I.phiA = before[i].phiA;
            I.phiB = before[i].phiB;
            I.u = before[i].u;
            I.ut = before[i].ut;
            I.step = before[i].step;
        }
    return st;
}

etd_status capture_grouped_steps(etd_plan* plan, ScheduleState::Captured* out) {
    ScheduleState& S = plan->sched;
    std::vector<LaunchRecorder> rec;
    etd_status st = record_two_steps(plan, rec);
    if (st != ETD_OK) return st;
    // groups of instances with equal launch sequences, in order of first appearance
    std::vector<std::vector<int>> groups;
    {
        std::map<std::string, int> index;
        for (size_t i = 0; i < rec.size(); ++i) {
            for (const LaunchRecord& op : rec[i].ops)
                if (op.grid.y != 1 || op.grid.z != 1 || op.block.y != 1 || op.block.z != 1)
                    return fail(&plan->err, ETD_E_STATE, "grouped schedule: a recorded launch is not one-dimensional");
            const auto it = index.emplace(launch_signature(rec[i]), (int)groups.size()).first;
            if (it->second == (int)groups.size()) groups.emplace_back();
            groups[it->second].push_back((int)i);
        }
    }
    // the argument table: per group and pass, the instances' records side by side
    constexpr size_t kAlign = 256;
    std::vector<std::vector<size_t>> offset(groups.size());
    size_t total = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const LaunchRecorder& r0 = rec[groups[gi][0]];
        for (const LaunchRecord& op : r0.ops) {
            offset[gi].push_back(total);
            total += (op.args.size() * groups[gi].size() + kAlign - 1) & ~(kAlign - 1);
        }
    }
    std::vector<unsigned char> host(std::max<size_t>(total, 1), 0);
    for (size_t gi = 0; gi < groups.size(); ++gi)
        for (size_t p = 0; p < offset[gi].size(); ++p)
            for (size_t m = 0; m < groups[gi].size(); ++m) {
                // records at the array stride of the twin's tab[blockIdx.y]: sizeof the
                // argument record (a multiple of its alignment; the base is 256-aligned)
                const LaunchRecord& op = rec[groups[gi][m]].ops[p];
                std::memcpy(host.data() + offset[gi][p] + m * op.args.size(), op.args.data(), op.args.size());
            }
    void* table = nullptr;
    if (hipMalloc(&table, host.size()) != hipSuccess)
        return fail(&plan->err, ETD_E_NOMEM, "grouped schedule: no memory for the argument table");
    auto bail = [&](etd_status e) {
        (void)hipFree(table);
        return e;
    };
    if (hipError_t e = hipMemcpy(table, host.data(), host.size(), hipMemcpyHostToDevice); e != hipSuccess)
        return bail(fail(&plan->err, ETD_E_HIP, std::string("grouped schedule: table upload: ") + hipGetErrorString(e)));
    for (const LaunchRecorder& r : rec)
        for (const LaunchRecord& op : r.ops)
            (void)hipFuncSetAttribute(op.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)op.smem);
    const int nb = std::max(1, std::min(S.branches, (int)groups.size()));
    if ((st = ensure_branches(plan, nb)) != ETD_OK) return bail(st);
    hipStream_t s = S.cap;
    if (hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed); e != hipSuccess)
        return bail(fail(&plan->err, ETD_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e)));
    hipError_t e = hipEventRecord(S.fork, s);
    for (int b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(S.side[b], S.fork, 0);
    for (size_t gi = 0; gi < groups.size() && e == hipSuccess; ++gi) {
        const LaunchRecorder& r0 = rec[groups[gi][0]];
        const unsigned m = (unsigned)groups[gi].size();
        for (size_t p = 0; p < r0.ops.size() && e == hipSuccess; ++p) {
            const LaunchRecord& op = r0.ops[p];
            void* tab = static_cast<char*>(table) + offset[gi][p];
            void* args[] = {&tab};
            e = hipLaunchKernel(op.fn, dim3(op.grid.x, m, 1), op.block, args, op.smem, S.side[gi % nb]);
        }
    }
    for (int b = 0; b < nb && e == hipSuccess; ++b) {
        e = hipEventRecord(S.join[b], S.side[b]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, S.join[b], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = ee;
    if (e == hipSuccess) e = hipGraphInstantiateWithFlags(&out->exec, graph, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return bail(fail(&plan->err, ETD_E_HIP, std::string("grouped schedule: capture: ") + hipGetErrorString(e)));
    out->table = table;
    size_t launches = 0;
    for (const auto& gr : groups) launches += rec[gr[0]].ops.size();
    log_msg(2, "plan %p: grouped %zu instance(s) into %zu group(s), %zu launches per two steps on %d branch(es)",
            (void*)plan, plan->inst.size(), groups.size(), launches, nb);
    return ETD_OK;
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
    if ((mode != ETD_EXEC_EAGER && mode != ETD_EXEC_GRAPH && mode != ETD_EXEC_GROUPED) || branches < 1 ||
        branches > 64)
        return false;
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
    bool tables = false;
    for (const auto& kv : plan->sched.graphs) tables |= kv.second.table != nullptr;
    if (tables) (void)hipStreamSynchronize(plan->stream);   // a replay in flight reads its table
    for (auto& kv : plan->sched.graphs) {
        (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.table) (void)hipFree(kv.second.table);
    }
    plan->sched.graphs.clear();
}

void etd::release_schedule(etd_plan* plan) {
    drop_graphs(plan);
    ScheduleState& S = plan->sched;
    for (hipStream_t st : S.side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : S.join) (void)hipEventDestroy(e);
    if (S.fork) (void)hipEventDestroy(S.fork);
    if (S.cap) (void)hipStreamDestroy(S.cap);
    if (S.rec) (void)hipStreamDestroy(S.rec);
    S.rec = nullptr;
    S.side.clear();
    S.join.clear();
    S.fork = nullptr;
    S.cap = nullptr;
}

etd_status etd::run_steps(etd_plan* plan, int nsteps) {
    ScheduleState& S = plan->sched;
    bool host_checks = false;   // the band solve reads its convergence flag on the host
    for (const Instance& I : plan->inst) host_checks |= (I.d.flags & ETD_F_SURFACE_NONLOCAL) != 0;
    if (S.mode == ETD_EXEC_EAGER || plan->timing || host_checks) return eager_steps(plan, nsteps);
    int k = 0;
    for (; k + 2 <= nsteps; k += 2) {
        const std::string key = graph_key(plan);
        auto it = S.graphs.find(key);
        if (it == S.graphs.end()) {
            const std::string before = pointer_state(plan);
            ScheduleState::Captured cap;
            etd_status st = S.mode == ETD_EXEC_GROUPED ? capture_grouped(plan, &cap) : capture_two_steps(plan, &cap.exec);
            if (st != ETD_OK) return st;
            if (pointer_state(plan) != before) {   // the replay would not match the host state
                (void)hipGraphExecDestroy(cap.exec);
                if (cap.table) (void)hipFree(cap.table);
                return fail(&plan->err, ETD_E_STATE, "graph schedule: the step state does not repeat after two steps");
            }
            it = S.graphs.emplace(key, cap).first;
        } else {
            for (Instance& I : plan->inst) I.step += 2;
        }
        HIPCHK(plan, hipGraphLaunch(it->second.exec, plan->stream));
    }
    return eager_steps(plan, nsteps - k);
}

extern "C" {

etd_status etd_set_schedule(etd_plan_t plan, const etd_schedule* sched) {
    if (!plan || !sched) return fail(plan ? &plan->err : nullptr, ETD_E_ARG, "null argument");
    if (sched->mode != ETD_EXEC_EAGER && sched->mode != ETD_EXEC_GRAPH && sched->mode != ETD_EXEC_GROUPED)
        return fail(&plan->err, ETD_E_ARG, "schedule mode must be ETD_EXEC_EAGER, ETD_EXEC_GRAPH or ETD_EXEC_GROUPED");
    if (sched->branches < 1 || sched->branches > 64)
        return fail(&plan->err, ETD_E_ARG, "schedule branches must be in 1..64");
    if (sched->xlines != 0 && sched->xlines != 8 && sched->xlines != 16)
        return fail(&plan->err, ETD_E_ARG, "schedule xlines must be 0, 8 or 16");
    if (sched->mode == ETD_EXEC_GROUPED)
        for (size_t i = 0; i < plan->inst.size(); ++i)
            if (!groupable(plan->inst[i]))
                return fail(&plan->err, ETD_E_ARG,
                            "grouped schedule: instance " + std::to_string(i) +
                                " is not a coupled 3D instance without band, diagnostics ring, mass projection and "
                                "band solve");
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
                                                   {ETD_EXEC_GRAPH, 32, 0}, {ETD_EXEC_GROUPED, 1, 0},
                                                   {ETD_EXEC_GROUPED, 8, 0}, {ETD_EXEC_EAGER, 1, 8}};
    bool tile_knob = false, all_groupable = true;
    for (const Instance& I : plan->inst) {
        tile_knob = tile_knob || (I.d.model == ETD_COUPLED && I.f32 && I.g.nx > 1);
        all_groupable = all_groupable && groupable(I);
    }
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
        if (cand[c].mode == ETD_EXEC_GROUPED && (!all_groupable || (cand[c].branches > 1 && ninst < 2))) continue;
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
