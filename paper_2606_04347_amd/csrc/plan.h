// Plan and instance state shared by the C-ABI entry points (api.hip) and
// the step schedules (schedule.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "etd.h"
#include "fft.h"
#include "kernels.h"

namespace etd {

// Last error message of any plan (etd_last_error(NULL)).
extern std::string g_last_error;

// Record msg as the last error (and in *sink) and return st; with ETD_LOG >= 1
// the message also goes to stderr.
etd_status fail(std::string* sink, etd_status st, const std::string& msg);

// Host logging to stderr.  ETD_LOG, read once per process: 0 (default) quiet,
// 1 errors, 2 also plan creation, graph captures and autotuner decisions.
int log_level();
void log_msg(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// A roctx range (rocprofv3 --marker-trace) around one stage of a step on the
// host: it spans the enqueue of the stage's kernels (under graph capture, the
// capture).  ETD_ROCTX=0 turns the ranges off.
class StageRange {
  public:
    explicit StageRange(const char* name);
    ~StageRange();
    StageRange(const StageRange&) = delete;
    StageRange& operator=(const StageRange&) = delete;

  private:
    bool on_;
};

// device scalar slots
enum Slot {
    S_INTPHI = 0, S_MASS = 1, S_Q0 = 2, S_MPS = 3 /* 2 values */, S_TMP = 5,
    S_DIAG = 8 /* 7 */, S_ENERGY = 16 /* 7 */, S_GERSH = 24, S_ABS = 25,
    S_HALT = 26 /* 1 once a non-finite value was seen: later steps are no-ops */, S_COUNT = 32
};

struct Instance {
    etd_instance_desc d{};
    etd_coupled_params cp{};
    etd_fixed_params fp{};
    GridK g{};
    bool f32 = false;
    std::vector<void*> allocs;
    size_t bytes = 0;
    FFTTables<float> tf;
    FFTTables<double> td;
    // coupled buffers (element type float or double)
    void *phiA = nullptr, *phiB = nullptr, *u = nullptr, *ut = nullptr, *lap = nullptr, *gx = nullptr,
         *gy = nullptr, *gz = nullptr, *P = nullptr, *Q = nullptr, *gp = nullptr, *vx = nullptr, *vy = nullptr,
         *vz = nullptr, *psi = nullptr;
    void *Sphi = nullptr, *St = nullptr, *Sra = nullptr, *Sa = nullptr, *Sb = nullptr, *Sgu = nullptr,
         *Stmp = nullptr;
    // fixed buffers (double unless noted)
    double *G = nullptr, *sg = nullptr, *isg = nullptr, *U = nullptr, *w = nullptr, *R0 = nullptr,
           *vv = nullptr, *t1 = nullptr, *t2 = nullptr, *acc = nullptr, *q = nullptr, *mq = nullptr,
           *t3 = nullptr, *t4 = nullptr,   // two-term recurrence passes (3D grids)
           *psid = nullptr;
    float *qf = nullptr, *psif = nullptr;   // FP32-FFT variant of the nonlocal term
    double* gf = nullptr;   // operator field: G, or for ETD_F_BAND_STEP g on the band and -1 off it
    // shared
    uint8_t* mask = nullptr;
    int32_t* band_idx = nullptr;
    int64_t* band_cnt = nullptr;   // band_blocks + 1 entries, then the total
    int64_t* band_total = nullptr;
    double* scal = nullptr;
    double* part = nullptr;
    double* fd = nullptr;          // per-axis FD symbol tables 4/h^2 sin^2(pi i / N)
    CoupledK K{};
    FixedK FK{};
    double A0 = 0.0;
    long step = 0;
    bool has_state = false;
    bool band_active = false;
    // fixed-model constants
    double C = 0, Bmbp = 0, Bes = 0, rho = 0, a = 0, b = 0;
    std::vector<double> ch1, ch2;   // Chebyshev coefficients of phi1(tau x), phi2(tau x) on [a, b]
    // band solve of (-Delta_S,h)^{-1} (ETD_F_SURFACE_NONLOCAL, etd_surface_lapinv)
    void* surf = nullptr;
    SurfaceWork sw;
    SurfaceResult surf_last;
    // per-step diagnostics ring (etd_diag_ring_enable): ring_cap entries of
    // kDiagRingFields doubles; ring_meta = {entries pushed, step before the first}
    double* ring = nullptr;
    int ring_cap = 0;
    int xlines = 0;   // FP32 ETD x pass tile of this instance (the plan's schedule)
    int64_t* ring_meta = nullptr;
};


// Event pairs around FFT pass launches (etd_pass_timing).
struct EventHook : PassHook {
    struct Rec {
        int kind;
        double bytes;
        hipEvent_t e0, e1;
    };
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Rec> recs;
    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    hipEvent_t pending = nullptr;
    void begin(int, hipStream_t s) override {
        pending = take();
        if (pending) (void)hipEventRecord(pending, s);
    }
    void end(int kind, double bytes, hipStream_t s) override {
        hipEvent_t e1 = take();
        if (!pending || !e1) return;
        (void)hipEventRecord(e1, s);
        recs.push_back({kind, bytes, pending, e1});
        pending = nullptr;
    }
    void reset() {
        used = 0;
        recs.clear();
        pending = nullptr;
    }
    ~EventHook() override {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// Execution schedule of etd_step (etd_schedule) with its HIP graph cache.
struct ScheduleState {
    int mode = 0;       // etd_exec_mode
    int branches = 1;
    int xlines = 0;     // FP32 ETD x pass tile: 0 (default) or 8 lines
    hipStream_t cap = nullptr;         // capture origin (default priority)
    std::vector<hipStream_t> side;     // capture branches (default priority)
    std::vector<hipEvent_t> join;      // one per branch
    hipEvent_t fork = nullptr;
    hipStream_t rec = nullptr;         // the grouped schedule's recording stream (default priority)
    // captured graphs keyed by pointer state and band-rebuild pattern; a
    // grouped graph also owns the device table of its launches' arguments
    struct Captured {
        hipGraphExec_t exec = nullptr;
        void* table = nullptr;
    };
    std::map<std::string, Captured> graphs;
};

// One step of one instance, enqueued on stream s (api.hip).
etd_status step_instance(etd_plan* plan, Instance& I, hipStream_t s);
// etd_step under the plan's schedule (schedule.hip).
etd_status run_steps(etd_plan* plan, int nsteps);
// Drop the captured graphs (after set_state or a schedule change) / release everything.
void drop_graphs(etd_plan* plan);
void release_schedule(etd_plan* plan);
// Device buffers (address, bytes) whose contents a step carries over to the
// next one, besides the host-side step counter and A0 (schedule.hip): what a
// snapshot or a checkpoint holds.  The fields computed from g alone (fixed
// model) and the buffers every step writes before it reads them are not
// among them.
std::vector<std::pair<void*, size_t>> carried_state(const Instance& I);

}  // namespace etd

struct etd_plan {
    std::vector<etd::Instance> inst;
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    etd::EventHook hook;
    bool timing = false;
    etd::ScheduleState sched;
};



#define HIPCHK(plan, call)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return etd::fail(plan ? &plan->err : nullptr, ETD_E_HIP,                                    \
                             std::string(#call) + ": " + hipGetErrorString(e_));                        \
    } while (0)
