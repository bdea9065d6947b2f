// server.hip -- served Poisson solves: requests arrive over time, are admitted
// when their whole device footprint fits the budget, keep their CG state
// resident, and advance together: a CG iteration of every admitted solve, of
// any degree and precision, is one merged operator launch (plus one for the
// small FP64 solves that take the one-thread-per-node operator, and one for
// degrees above 11) and one assemble-update launch.  A solve's workgroups do
// exactly what its own launch would do (per-solve partials, reductions and
// tickets), so its result does not depend on which other solves share the
// launches.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "nek_internal.h"

extern "C" int nek_box_numbering(int Ex, int Ey, int Ez, int N, int64_t *glo, uint8_t *dirichlet);

namespace nek {
namespace {

constexpr int MAX_SLOTS = 64;
static_assert(MAX_SLOTS <= BATCH_MAX_SLOTS, "a batched launch holds at most BATCH_MAX_SLOTS solves");
constexpr int PREP_THREADS = 4;   // host threads preparing submitted requests

bool f32_operator(int prec) { return prec == NEK_PREC_F32G32 || prec == NEK_PREC_F32GBF16; }
bool is_mixed(int prec) { return f32_operator(prec) || prec == NEK_PREC_F64G32 || prec == NEK_PREC_F64GBF16; }
int g_storage(int prec) { return prec == NEK_PREC_F32G32 || prec == NEK_PREC_F64G32 ? NEK_G_F32 : NEK_G_BF16; }

// Device bytes of one admitted request (arena + solution vector).  The
// gather-scatter part is bounded by one int32 per local point plus two bit
// sets (first copies; copies of shared or masked nodes): every local point
// appears in at most one group.
struct Footprint {
    size_t g, b, gs, D, D32, glo, ws, arena, x, total;
};

Footprint footprint_of(int64_t E, int N, int prec) {
    const size_t P = (size_t)(E * n3_of(N));
    const size_t n2 = (size_t)(N + 1) * (N + 1);
    Footprint f;
    f.g = align256(6 * P * sizeof(double));
    f.b = align256(P * sizeof(double));
    f.gs = align256(P * sizeof(int32_t) + 4) + 2 * align256((P + 31) / 32 * sizeof(uint32_t));
    f.D = align256(n2 * sizeof(double));
    f.D32 = align256(n2 * sizeof(float));
    f.glo = !is_mixed(prec) ? 0
          : g_storage(prec) == NEK_G_F32 ? align256(6 * P * sizeof(float)) : align256(6 * P * sizeof(uint16_t));
    f.ws = cg_layout(E, N, 0).total;
    f.arena = f.g + f.b + f.gs + f.D + f.D32 + f.glo + f.ws;
    f.x = align256(P * sizeof(double));
    f.total = f.arena + f.x;
    return f;
}

struct Request {
    uint64_t id = 0;
    nek_request spec{};
    bool mesh = false;            // the caller's own D, g, glo, dirichlet (else a box)
    bool on_device = false;       // the caller's arrays are device memory
    int64_t E = 0, P = 0;
    Footprint fp{};
    double t_submit = 0.0;
    // filled by the preparation thread
    std::atomic<bool> prepared{false};
    int prep_status = NEK_OK;
    std::string prep_msg;
    GsHost gs;                    // group metadata; index arrays dropped once staged
    // pinned: b (host b) | gs idx | own bits | rowed bits | D | D32 | g (host g of a mesh)
    void *staging = nullptr;
    size_t staging_bytes = 0;
    size_t off_b = 0, off_idx = 0, off_own = 0, off_rowed = 0, off_D = 0, off_D32 = 0, off_g = 0;
};

// Pinned host buffers, reused once their upload has completed.
struct PinnedPool {
    struct Buf {
        void *p;
        size_t n;
        bool busy;
    };
    std::mutex mu;
    std::vector<Buf> bufs;
    void *get(size_t n) {
        {
            std::lock_guard<std::mutex> lk(mu);
            size_t best = (size_t)-1;
            for (size_t i = 0; i < bufs.size(); ++i)
                if (!bufs[i].busy && bufs[i].n >= n && (best == (size_t)-1 || bufs[i].n < bufs[best].n)) best = i;
            if (best != (size_t)-1) {
                bufs[best].busy = true;
                return bufs[best].p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> lk(mu);
        bufs.push_back({p, n, true});
        return p;
    }
    void put(void *p) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &b : bufs)
            if (b.p == p) b.busy = false;
    }
    void release_all() {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &b : bufs) (void)hipHostFree(b.p);
        bufs.clear();
    }
};

enum SlotState { ACTIVE, FINISHING, DONE };

struct FinArea {        // pinned landing area of a finishing solve
    CgScalars sc;
    double t2;
};

struct Slot {
    std::unique_ptr<Request> req;
    int index = -1;               // 0..MAX_SLOTS-1, for the pinned finishing area
    SlotState state = ACTIVE;
    char *arena = nullptr;
    double *x = nullptr;
    double *g = nullptr, *b = nullptr, *D = nullptr;
    float *D32 = nullptr;
    void *glo = nullptr;
    CgWs W{};
    GsDevice gsd;
    int replacements = 0;
    double t_admit = 0.0, t_done = 0.0;
    hipEvent_t ev_upload = nullptr;
    hipEvent_t ev_fin = nullptr;
    nek_result res{};
};

struct TableSet {       // slot tables of one step, host (pinned) and device
    char *host = nullptr;
    char *dev = nullptr;
    hipEvent_t ev = nullptr;     // after the last work that read this set
    bool used = false;
};

// Iterations per server iteration: a solve of weight w takes part in the
// first w of up to MAX_ITER_WEIGHT rounds of launches, so small solves do not
// move at the pace of the largest ones.  A solve's iteration costs about its
// local points; a round of launches about LAUNCH_POINTS more (its fixed
// launch and reduction latency).  A solve gets weight min(8, cmax / (2 P))
// (cmax the costliest solve), and the top levels are dropped until the extra
// rounds cost at most half of the first one.
constexpr int64_t LAUNCH_POINTS = 500000;
constexpr int MAX_ITER_WEIGHT = 8;

int assign_weights(const std::vector<int64_t> &points, std::vector<int> &wt) {
    const size_t n = points.size();
    wt.assign(n, 1);
    if (n < 2) return 1;
    int64_t cmax = 0, total = 0;
    for (int64_t p : points) {
        cmax = std::max(cmax, p);
        total += p;
    }
    int wmax = 1;
    for (size_t i = 0; i < n; ++i) {
        const int64_t w = cmax / (2 * std::max<int64_t>(points[i], 1));
        wt[i] = (int)std::min<int64_t>(MAX_ITER_WEIGHT, std::max<int64_t>(1, w));
        wmax = std::max(wmax, wt[i]);
    }
    const int64_t budget = (total + LAUNCH_POINTS) / 2;
    for (; wmax > 1; --wmax) {
        int64_t extra = 0;
        for (int j = 1; j < wmax; ++j) {
            extra += LAUNCH_POINTS;
            for (size_t i = 0; i < n; ++i)
                if (std::min(wt[i], wmax) > j) extra += points[i];
        }
        if (extra <= budget) break;
    }
    for (int &w : wt) w = std::min(w, wmax);
    return wmax;
}

// One of the launches of a round: its table (slots in weight order, so the
// solves of round j are a prefix of it) and, per round, the prefix's slot
// count, workgroups and LDS.
struct LaunchPlan {
    int count[MAX_ITER_WEIGHT] = {};
    int64_t blocks[MAX_ITER_WEIGHT] = {};
    size_t lds[MAX_ITER_WEIGHT] = {};
};

constexpr size_t TABLE_BYTES =
    MAX_SLOTS * (2 * sizeof(ServeAxSlot) + 2 * sizeof(ServeNodeSlot) + sizeof(AsmSlot) + sizeof(CgScalars *));

}  // namespace
}  // namespace nek

using namespace nek;

struct nek_server {
    size_t budget = 0;
    size_t used = 0;
    int device = 0;                                   // the device the server runs on
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr;
    std::chrono::steady_clock::time_point t0;
    uint64_t next_id = 1;

    // preparation threads: requests are prepared independently, admitted in
    // arrival order
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> prep_queue;
    bool stop = false;
    PinnedPool pinned;

    std::deque<std::unique_ptr<Request>> waiting;     // arrival order
    std::vector<std::unique_ptr<Slot>> slots;         // admitted (ACTIVE / FINISHING)
    std::map<uint64_t, std::unique_ptr<Slot>> done;   // finished, solution not fetched
    std::deque<nek_result> results;                   // finished, not reported
    std::vector<int> free_index;

    // tables
    TableSet tables[2];
    int cur_table = 0;
    bool dirty = true;
    // the launches of a round: the two merged pencil operators, the two
    // node operators (n = 9 apart), the assemble-update
    enum { L_PEN, L_PEN_HI, L_NODE, L_NODE9, L_ASM, N_LAUNCH };
    LaunchPlan plan[N_LAUNCH];
    int wmax = 1;
    std::vector<Slot *> table_slots;                  // slots of the current tables, in order
    // status snapshots, one step behind
    CgScalars *status_dev[2] = {nullptr, nullptr};
    CgScalars *status_host[2] = {nullptr, nullptr};
    hipEvent_t ev_status[2] = {nullptr, nullptr};
    std::vector<Slot *> status_slots[2];
    bool status_pending[2] = {false, false};
    int status_parity = 0;
    FinArea *fin = nullptr;                           // pinned, MAX_SLOTS

    double clock() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // ------------------------------------------------------------ preparation
    // Numbering and gather-scatter tables on the host, then everything the
    // admission uploads into pinned staging.  A mesh of the caller's own in
    // device memory comes to the host on this thread's stream (glo,
    // dirichlet, D); its b and g are copied device to device at admission.
    void prepare(Request *R, hipStream_t ps) {
        const nek_request &q = R->spec;
        const int64_t P = R->P;
        const int n = q.N + 1;
        std::vector<int64_t> glo;
        std::vector<uint8_t> dr;
        double D[(NEK_MAX_DEGREE + 1) * (NEK_MAX_DEGREE + 1)];
        const int64_t *glo_p = q.glo;
        const uint8_t *dir_p = q.dirichlet;
        R->prep_status = NEK_OK;
        if (!R->mesh) {
            glo.resize((size_t)P);
            dr.resize((size_t)P);
            nek_box_numbering(q.Ex, q.Ey, q.Ez, q.N, glo.data(), dr.data());
            glo_p = glo.data();
            dir_p = dr.data();
            gll_host(q.N, nullptr, nullptr, D);
        } else if (R->on_device) {
            glo.resize((size_t)P);
            hipError_t e = hipMemcpyAsync(glo.data(), q.glo, (size_t)P * sizeof(int64_t), hipMemcpyDeviceToHost, ps);
            if (e == hipSuccess && q.dirichlet) {
                dr.resize((size_t)P);
                e = hipMemcpyAsync(dr.data(), q.dirichlet, (size_t)P, hipMemcpyDeviceToHost, ps);
            }
            if (e == hipSuccess) e = hipMemcpyAsync(D, q.D, (size_t)n * n * sizeof(double), hipMemcpyDeviceToHost, ps);
            if (e == hipSuccess) e = hipStreamSynchronize(ps);
            if (e != hipSuccess) {
                R->prep_status = NEK_ERR_DEVICE;
                R->prep_msg = std::string("copying the request's numbering and D to the host: ") + hipGetErrorString(e);
            }
            glo_p = glo.data();
            dir_p = q.dirichlet ? dr.data() : nullptr;
        } else {
            memcpy(D, q.D, (size_t)n * n * sizeof(double));
        }
        if (R->prep_status == NEK_OK)
            R->prep_status = gs_build_host(R->E, q.N, glo_p, dir_p, true, R->gs, R->prep_msg);
        if (R->prep_status == NEK_OK) {
            const bool host_b = !R->on_device, host_g = R->mesh && !R->on_device;
            size_t at = 0;
            R->off_b = at;
            if (host_b) at += align256((size_t)P * sizeof(double));
            R->off_idx = at;
            at += align256(R->gs.idx.size() * sizeof(int32_t) + 4);
            R->off_own = at;
            at += align256(R->gs.own.size() * sizeof(uint32_t));
            R->off_rowed = at;
            at += align256(R->gs.rowed.size() * sizeof(uint32_t));
            R->off_D = at;
            at += align256((size_t)n * n * sizeof(double));
            R->off_D32 = at;
            at += align256((size_t)n * n * sizeof(float));
            R->off_g = at;
            if (host_g) at += align256((size_t)6 * P * sizeof(double));
            R->staging_bytes = at;
            R->staging = pinned.get(R->staging_bytes);
            if (!R->staging) {
                R->prep_status = NEK_ERR_NOMEM;
                R->prep_msg = "pinned staging allocation failed";
            } else {
                char *st = (char *)R->staging;
                if (host_b) memcpy(st + R->off_b, q.b, (size_t)P * sizeof(double));   // the caller's b, read once
                if (!R->gs.idx.empty()) memcpy(st + R->off_idx, R->gs.idx.data(), R->gs.idx.size() * sizeof(int32_t));
                memcpy(st + R->off_own, R->gs.own.data(), R->gs.own.size() * sizeof(uint32_t));
                memcpy(st + R->off_rowed, R->gs.rowed.data(), R->gs.rowed.size() * sizeof(uint32_t));
                memcpy(st + R->off_D, D, (size_t)n * n * sizeof(double));
                float *D32 = (float *)(st + R->off_D32);
                for (int t = 0; t < n * n; ++t) D32[t] = (float)D[t];
                if (host_g) memcpy(st + R->off_g, q.g, (size_t)6 * P * sizeof(double));
            }
        }
        R->prepared.store(true, std::memory_order_release);
    }

    void worker_loop() {
        (void)hipSetDevice(device);
        hipStream_t ps = nullptr;
        const bool have_stream = hipStreamCreateWithFlags(&ps, hipStreamNonBlocking) == hipSuccess;
        for (;;) {
            Request *R = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !prep_queue.empty(); });
                if (stop) break;
                R = prep_queue.front();
                prep_queue.pop_front();
            }
            if (!have_stream && R->mesh && R->on_device) {
                R->prep_status = NEK_ERR_DEVICE;
                R->prep_msg = "no stream for the preparation thread";
                R->prepared.store(true, std::memory_order_release);
                continue;
            }
            prepare(R, ps);
        }
        if (have_stream) (void)hipStreamDestroy(ps);
    }

    // ------------------------------------------------------------ admission
    // A request that could not be prepared or admitted is reported as finished
    // with that status; its staging buffer goes back to the pool.
    void report_failed(Request &R, int status) {
        nek_result r{};
        r.id = R.id;
        r.status = status;
        r.t_submit = R.t_submit;
        r.t_admit = r.t_done = clock();
        r.E = R.E;
        r.N = R.spec.N;
        if (R.staging) pinned.put(R.staging);
        R.staging = nullptr;
        results.push_back(r);
    }

    int admit_one(std::unique_ptr<Request> R) {
        const nek_request &q = R->spec;
        const Footprint &f = R->fp;
        auto S = std::make_unique<Slot>();
        S->index = free_index.back();
        free_index.pop_back();
        hipError_t e = hipMallocAsync((void **)&S->arena, f.arena, stream);
        if (e == hipSuccess) e = hipMallocAsync((void **)&S->x, f.x, stream);
        if (e == hipErrorOutOfMemory) {
            // the device is short of memory although the budget is not: report
            // the request as failed and keep serving the others
            if (S->arena) (void)hipFreeAsync(S->arena, stream);
            free_index.push_back(S->index);
            report_failed(*R, NEK_ERR_NOMEM);
            return NEK_OK;
        }
        if (e != hipSuccess) return check_hip(e, "server admission: hipMallocAsync");
        char *a = S->arena;
        S->g = (double *)a;
        a += f.g;
        S->b = (double *)a;
        a += f.b;
        char *gs_arena = a;
        a += f.gs;
        S->D = (double *)a;
        a += f.D;
        S->D32 = (float *)a;
        a += f.D32;
        S->glo = f.glo ? (void *)a : nullptr;
        a += f.glo;
        S->W = cg_ws(a, R->E, q.N, 0);
        // uploads (pinned staging, or the caller's device arrays) and device
        // setup, all on the server stream
        const char *st = (const char *)R->staging;
        // b arrives in the layout of Listing 1 (through w) and is kept in the CG layout
        if (R->on_device)
            NEK_HIP(hipMemcpyAsync(S->W.w, q.b, (size_t)R->P * sizeof(double), hipMemcpyDeviceToDevice, stream));
        else
            NEK_HIP(hipMemcpyAsync(S->W.w, st + R->off_b, (size_t)R->P * sizeof(double), hipMemcpyHostToDevice,
                                   stream));
        NEK_HIP(launch_permute(R->E, q.N, S->W.w, S->b, true, stream));
        const size_t own_off = R->gs.idx_bytes();   // == off_own - off_idx
        NEK_HIP(hipMemcpyAsync(gs_arena, st + R->off_idx, own_off, hipMemcpyHostToDevice, stream));
        NEK_HIP(hipMemcpyAsync(gs_arena + own_off + R->gs.own_bytes(), st + R->off_rowed,
                               R->gs.rowed.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
        NEK_HIP(hipMemcpyAsync(gs_arena + own_off, st + R->off_own, R->gs.own.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, stream));
        const size_t n2 = (size_t)(q.N + 1) * (q.N + 1);
        NEK_HIP(hipMemcpyAsync(S->D, st + R->off_D, n2 * sizeof(double), hipMemcpyHostToDevice, stream));
        NEK_HIP(hipMemcpyAsync(S->D32, st + R->off_D32, n2 * sizeof(float), hipMemcpyHostToDevice, stream));
        if (R->mesh)
            NEK_HIP(hipMemcpyAsync(S->g, R->on_device ? (const void *)q.g : (const void *)(st + R->off_g),
                                   (size_t)6 * R->P * sizeof(double),
                                   R->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, stream));
        NEK_HIP(hipEventCreateWithFlags(&S->ev_upload, hipEventDisableTiming));
        NEK_HIP(hipEventRecord(S->ev_upload, stream));
        gs_attach(R->gs, gs_arena, S->gsd);
        std::vector<int32_t>().swap(R->gs.idx);
        std::vector<uint32_t>().swap(R->gs.own);
        std::vector<uint32_t>().swap(R->gs.rowed);
        if (!R->mesh) {
            GllTable tab;
            memset(&tab, 0, sizeof(tab));
            gll_host(q.N, tab.z, tab.w, tab.D);
            NEK_HIP(launch_box_geometry(q.Ex, q.Ey, q.Ez, q.N, q.amp, q.a[0], q.a[1], q.a[2], tab, S->g,
                                        nullptr, nullptr, stream));
        }
        if (is_mixed(q.precision))
            NEK_HIP(launch_convert_g(R->E, q.N, S->g, g_storage(q.precision), S->glo, stream));
        const double drop = is_mixed(q.precision) ? reliable_drop_default(q.precision) : 0.0;
        NEK_HIP(launch_cg_reset(S->W.sc, S->W.tickets, N_SITES * RED_TICKETS, q.max_iter, q.rel_tol, drop,
                                stream));
        NEK_HIP(launch_cg_init(R->P, S->b, S->x, S->W.r, S->W.p, S->gsd.own_bits, nullptr, S->W.site(SITE_INIT),
                               S->W.sc, stream));
        used += f.total;
        S->t_admit = clock();
        S->res.id = R->id;
        S->res.t_submit = R->t_submit;
        S->res.t_admit = S->t_admit;
        S->res.E = R->E;
        S->res.N = q.N;
        S->res.footprint = f.total;
        S->req = std::move(R);
        slots.push_back(std::move(S));
        dirty = true;
        return NEK_OK;
    }

    // Admission in arrival order among prepared requests: a request still in
    // preparation does not hold back prepared ones behind it, but a prepared
    // request that does not fit stops admission, so a large request is never
    // overtaken indefinitely by smaller ones.
    int admit() {
        for (auto it = waiting.begin(); it != waiting.end();) {
            Request *R = it->get();
            if (!R->prepared.load(std::memory_order_acquire)) {
                ++it;
                continue;
            }
            if (R->prep_status != NEK_OK) {
                report_failed(*R, R->prep_status);
                it = waiting.erase(it);
                continue;
            }
            if (used + R->fp.total > budget || free_index.empty()) break;
            std::unique_ptr<Request> own = std::move(*it);
            it = waiting.erase(it);
            int rc = admit_one(std::move(own));
            if (rc != NEK_OK) return rc;
        }
        return NEK_OK;
    }

    // ------------------------------------------------------------ tables
    int rebuild_tables() {
        const int k = cur_table ^ 1;
        TableSet &T = tables[k];
        if (T.used) NEK_HIP(hipEventSynchronize(T.ev));   // its last reader has finished
        std::vector<Slot *> act;
        for (auto &s : slots)
            if (s->state == ACTIVE) act.push_back(s.get());
        std::vector<int64_t> pts;
        for (Slot *S : act) pts.push_back(S->req->P);
        std::vector<int> wt;
        wmax = assign_weights(pts, wt);
        // heaviest weight first: the solves of round j are those of weight > j
        std::vector<size_t> order(act.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return wt[a] > wt[b]; });
        ServeAxSlot *pen = (ServeAxSlot *)T.host;
        ServeAxSlot *pen_hi = pen + MAX_SLOTS;
        ServeNodeSlot *node = (ServeNodeSlot *)(pen_hi + MAX_SLOTS);
        ServeNodeSlot *node9 = node + MAX_SLOTS;
        AsmSlot *asl = (AsmSlot *)(node9 + MAX_SLOTS);
        CgScalars **scp = (CgScalars **)(asl + MAX_SLOTS);
        int cnt[N_LAUNCH] = {};
        int64_t blk[N_LAUNCH] = {};
        size_t lds[N_LAUNCH] = {};
        for (LaunchPlan &L : plan) L = LaunchPlan{};
        std::vector<Slot *> ordered;
        // close round j of every launch: the prefix so far is what it runs
        auto close_rounds = [&](int from, int to) {
            for (int j = from; j < to; ++j)
                for (int l = 0; l < N_LAUNCH; ++l) {
                    plan[l].count[j] = cnt[l];
                    plan[l].blocks[j] = blk[l];
                    plan[l].lds[j] = lds[l];
                }
        };
        int prev_w = MAX_ITER_WEIGHT;
        for (size_t oi = 0; oi < order.size(); ++oi) {
            const size_t i = order[oi];
            Slot *S = act[i];
            // rounds j >= wt[i] hold only the solves before this one
            if (wt[i] < prev_w) close_rounds(wt[i], prev_w);
            prev_w = wt[i];
            const nek_request &q = S->req->spec;
            const int64_t E = S->req->E;
            const bool mixed = is_mixed(q.precision);
            int64_t nparts;
            AxFuse fz;
            fz.r = S->W.r;
            fz.x = S->x;
            fz.partials = S->W.axp;
            fz.sc = S->W.sc;
            fz.cg_layout = true;
            // the operator nek_cg_solve would run (bitwise the same solve)
            if (!mixed && ax_node_fused_fits(E, q.N)) {
                ServeNodeShape sh;
                if (!serve_node_shape(q.N, E, sh)) return fail(NEK_ERR_STATE, "server: no node shape");
                const int l = sh.n9 ? L_NODE9 : L_NODE;
                ServeNodeSlot &A = (sh.n9 ? node9 : node)[cnt[l]++];
                A.block0 = blk[l];
                A.E = E;
                A.nx = q.N + 1;
                A.pad_ = 0;
                A.D = S->D;
                A.g = S->g;
                A.p = S->W.p;
                A.w = S->W.w;
                A.fz = fz;
                blk[l] += sh.blocks;
                lds[l] = std::max(lds[l], sh.lds_bytes);
                nparts = E;
            } else {
                ServeAxShape sh;
                if (!serve_ax_shape(q.N, q.precision, E, sh)) return fail(NEK_ERR_STATE, "server: no operator shape");
                const int l = sh.hi ? L_PEN_HI : L_PEN;
                ServeAxSlot &A = (sh.hi ? pen_hi : pen)[cnt[l]++];
                A.block0 = blk[l];
                A.E = E;
                A.nx = q.N + 1;
                A.precision = q.precision;
                A.D = f32_operator(q.precision) ? (const void *)S->D32 : (const void *)S->D;
                A.g = mixed ? (const void *)S->glo : (const void *)S->g;
                A.p = S->W.p;
                A.w = S->W.w;
                A.fz = fz;
                blk[l] += sh.blocks;
                lds[l] = std::max(lds[l], sh.lds_bytes);
                nparts = sh.nparts;
            }
            AsmSlot &U = asl[cnt[L_ASM]++];
            U.block0 = blk[L_ASM];
            U.nblocks = asm_blocks(S->gsd);
            U.P = S->req->P;
            U.args = S->gsd.args;
            U.rowed = S->gsd.rowed_bits;
            U.r = S->W.r;
            U.w = S->W.w;
            U.axparts = S->W.axp;
            U.nparts = nparts;
            U.red = S->W.site(SITE_UPDATE);
            U.sc = S->W.sc;
            U.w_f32 = f32_operator(q.precision) ? 1 : 0;   // the FP32 operator leaves w in FP32
            blk[L_ASM] += U.nblocks;
            scp[ordered.size()] = S->W.sc;
            ordered.push_back(S);
        }
        close_rounds(0, prev_w);
        NEK_HIP(hipMemcpyAsync(T.dev, T.host, TABLE_BYTES, hipMemcpyHostToDevice, stream));
        // the set in use until now may be rewritten once the work queued so far is done
        if (tables[cur_table].used) NEK_HIP(hipEventRecord(tables[cur_table].ev, stream));
        T.used = true;
        cur_table = k;
        table_slots = ordered;
        dirty = false;
        return NEK_OK;
    }

    // ------------------------------------------------------------ finishing
    // A solve that leaves ACTIVE must not be seen by a pending snapshot: it may
    // finish, be fetched and be freed before that snapshot is read.
    void forget_in_snapshots(Slot *S) {
        for (int k = 0; k < 2; ++k)
            for (auto &p : status_slots[k])
                if (p == S) p = nullptr;
    }

    // A x alone, on vectors in the CG layout
    static AxFuse plain_cg() {
        AxFuse f;
        f.cg_layout = true;
        return f;
    }

    int start_finish(Slot *S) {
        forget_in_snapshots(S);
        const nek_request &q = S->req->spec;
        const int64_t E = S->req->E, P = S->req->P;
        NEK_HIP(launch_cg_finish(P, S->x, S->W.p, S->W.sc, stream));
        NEK_HIP(launch_ax_f64(E, q.N, S->D, S->g, S->x, S->W.w, plain_cg(), stream));
        NEK_HIP(launch_gs(S->gsd, S->W.w, stream));
        NEK_HIP(launch_gdiff2(P, S->b, S->W.w, S->gsd.own_bits, S->W.site(SITE_RESID), S->W.scratch, stream));
        // x back to the layout of Listing 1 (through w)
        NEK_HIP(launch_permute(E, q.N, S->x, S->W.w, false, stream));
        NEK_HIP(hipMemcpyAsync(S->x, S->W.w, (size_t)P * sizeof(double), hipMemcpyDeviceToDevice, stream));
        NEK_HIP(hipMemcpyAsync(&fin[S->index].sc, S->W.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, stream));
        NEK_HIP(hipMemcpyAsync(&fin[S->index].t2, S->W.scratch, sizeof(double), hipMemcpyDeviceToHost, stream));
        NEK_HIP(hipEventCreateWithFlags(&S->ev_fin, hipEventDisableTiming));
        NEK_HIP(hipEventRecord(S->ev_fin, stream));
        S->state = FINISHING;
        dirty = true;
        return NEK_OK;
    }

    int replace_residual(Slot *S) {
        const nek_request &q = S->req->spec;
        const int64_t E = S->req->E, P = S->req->P;
        NEK_HIP(launch_cg_finish(P, S->x, S->W.p, S->W.sc, stream));
        NEK_HIP(launch_ax_f64(E, q.N, S->D, S->g, S->x, S->W.w, plain_cg(), stream));
        NEK_HIP(launch_gs(S->gsd, S->W.w, stream));
        NEK_HIP(launch_cg_replace(P, S->b, S->W.w, S->W.r, S->gsd.own_bits, S->W.site(SITE_REPLACE),
                                  S->W.sc, stream));
        S->replacements++;
        return NEK_OK;
    }

    void check_finishing() {
        for (size_t i = 0; i < slots.size();) {
            Slot *S = slots[i].get();
            bool moved = false;
            if (S->ev_upload && hipEventQuery(S->ev_upload) == hipSuccess) {
                (void)hipEventDestroy(S->ev_upload);
                S->ev_upload = nullptr;
                pinned.put(S->req->staging);
                S->req->staging = nullptr;
            }
            if (S->state == FINISHING && !S->ev_upload && hipEventQuery(S->ev_fin) == hipSuccess) {
                const nek_request &q = S->req->spec;
                const CgScalars &sc = fin[S->index].sc;
                const double bb = sc.bb;
                nek_result &r = S->res;
                r.iters = sc.it;
                r.n_replacements = sc.n_replace;
                r.rel_res = bb > 0.0 ? sqrt(sc.rr / bb) : 0.0;
                r.rel_res_true = bb > 0.0 ? sqrt(fin[S->index].t2 / bb) : 0.0;
                int status = sc.status;
                if (status == NEK_OK && q.rel_tol > 0.0) {
                    const double judged = is_mixed(q.precision) ? r.rel_res_true : r.rel_res;
                    if (!(judged <= q.rel_tol)) status = NEK_ERR_NOCONV;
                }
                r.status = status;
                r.t_done = clock();
                (void)hipEventDestroy(S->ev_fin);
                S->ev_fin = nullptr;
                (void)hipFreeAsync(S->arena, stream);
                S->arena = nullptr;
                used -= S->req->fp.arena;
                free_index.push_back(S->index);
                S->index = -1;
                S->state = DONE;
                forget_in_snapshots(S);
                results.push_back(r);
                done[r.id] = std::move(slots[i]);
                slots.erase(slots.begin() + (long)i);
                moved = true;
            }
            if (!moved) ++i;
        }
    }

    // ------------------------------------------------------------ one step
    int step(int iters, int *active, int *queued) {
        int rc = admit();
        if (rc != NEK_OK) return rc;
        if (dirty) {
            rc = rebuild_tables();
            if (rc != NEK_OK) return rc;
        }
        if (!table_slots.empty()) {
            const TableSet &T = tables[cur_table];
            const ServeAxSlot *pen = (const ServeAxSlot *)T.dev;
            const ServeAxSlot *pen_hi = pen + MAX_SLOTS;
            const ServeNodeSlot *node = (const ServeNodeSlot *)(pen_hi + MAX_SLOTS);
            const ServeNodeSlot *node9 = node + MAX_SLOTS;
            const AsmSlot *asl = (const AsmSlot *)(node9 + MAX_SLOTS);
            CgScalars *const *scp = (CgScalars *const *)(asl + MAX_SLOTS);
            // the host image of the same assembly slots, for launches that take them by value
            const AsmSlot *asl_host =
                (const AsmSlot *)((const ServeNodeSlot *)((const ServeAxSlot *)T.host + 2 * MAX_SLOTS) + 2 * MAX_SLOTS);
            const int base_iters = std::max(1, iters);
            for (int it = 0; it < base_iters; ++it) {
                for (int j = 0; j < wmax; ++j) {
                    const LaunchPlan &A = plan[L_PEN], &H = plan[L_PEN_HI], &V = plan[L_NODE], &V9 = plan[L_NODE9],
                                     &U = plan[L_ASM];
                    if (A.count[j]) NEK_HIP(launch_ax_serve(pen, A.count[j], A.blocks[j], A.lds[j], false, stream));
                    if (H.count[j]) NEK_HIP(launch_ax_serve(pen_hi, H.count[j], H.blocks[j], H.lds[j], true, stream));
                    if (V.count[j])
                        NEK_HIP(launch_ax_node_serve(node, V.count[j], V.blocks[j], V.lds[j], false, stream));
                    if (V9.count[j])
                        NEK_HIP(launch_ax_node_serve(node9, V9.count[j], V9.blocks[j], V9.lds[j], true, stream));
                    if (U.count[j] && U.count[j] <= ASM_KARG_SLOTS)
                        NEK_HIP(launch_assemble_update_batch_karg(asl_host, U.count[j], U.blocks[j], stream));
                    else if (U.count[j])
                        NEK_HIP(launch_assemble_update_batch(asl, U.count[j], U.blocks[j], stream));
                }
            }
            // snapshot of every active solve's scalars into buffer q; the snapshot
            // of the previous step (buffer q ^ 1) is inspected below, after this
            // step's work is queued, so the device stays busy while the host waits
            const int q = status_parity;
            NEK_HIP(launch_gather_scalars(scp, (int)table_slots.size(), status_dev[q], stream));
            NEK_HIP(hipMemcpyAsync(status_host[q], status_dev[q], table_slots.size() * sizeof(CgScalars),
                                   hipMemcpyDeviceToHost, stream));
            NEK_HIP(hipEventRecord(ev_status[q], stream));
            status_slots[q] = table_slots;
            status_pending[q] = true;
            status_parity ^= 1;
        }
        const int pq = status_parity;   // the buffer written one step before
        if (status_pending[pq]) {
            NEK_HIP(hipEventSynchronize(ev_status[pq]));
            status_pending[pq] = false;
            for (size_t i = 0; i < status_slots[pq].size(); ++i) {
                Slot *S = status_slots[pq][i];
                if (S == nullptr || S->state != ACTIVE) continue;
                const CgScalars &v = status_host[pq][i];
                if (v.done) {
                    rc = start_finish(S);
                    if (rc != NEK_OK) return rc;
                } else if (is_mixed(S->req->spec.precision) && v.need_replace && v.n_replace >= S->replacements) {
                    rc = replace_residual(S);
                    if (rc != NEK_OK) return rc;
                }
            }
        }
        check_finishing();
        if (active) {
            int a = 0;
            for (auto &s : slots)
                if (s->state == ACTIVE) ++a;
            *active = a;
        }
        if (queued) *queued = (int)waiting.size();
        return NEK_OK;
    }
};

extern "C" {

size_t nek_server_footprint(int Ex, int Ey, int Ez, int N, int precision) {
    if (Ex < 1 || Ey < 1 || Ez < 1 || N < 1 || N > NEK_MAX_DEGREE) return 0;
    return footprint_of((int64_t)Ex * Ey * Ez, N, precision).total;
}

size_t nek_server_footprint_mesh(int64_t E, int N, int precision) {
    if (E < 1 || N < 1 || N > NEK_MAX_DEGREE) return 0;
    return footprint_of(E, N, precision).total;
}

int nek_server_create(size_t hbm_budget, nek_server **out) {
    clear_error();
    if (!out) return fail(NEK_ERR_ARG, "nek_server_create: out is null");
    *out = nullptr;
    if (hbm_budget == 0) return fail(NEK_ERR_ARG, "nek_server_create: budget must be > 0");
    std::unique_ptr<nek_server> S(new nek_server());
    S->budget = hbm_budget;
    S->t0 = std::chrono::steady_clock::now();
    NEK_HIP(hipGetDevice(&S->device));
    NEK_HIP(hipStreamCreate(&S->stream));
    NEK_HIP(hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
        NEK_HIP(hipHostMalloc((void **)&S->tables[k].host, TABLE_BYTES, hipHostMallocDefault));
        NEK_HIP(hipMalloc((void **)&S->tables[k].dev, TABLE_BYTES));
        NEK_HIP(hipEventCreateWithFlags(&S->tables[k].ev, hipEventDisableTiming));
        NEK_HIP(hipMalloc((void **)&S->status_dev[k], MAX_SLOTS * sizeof(CgScalars)));
        NEK_HIP(hipHostMalloc((void **)&S->status_host[k], MAX_SLOTS * sizeof(CgScalars), hipHostMallocDefault));
        NEK_HIP(hipEventCreateWithFlags(&S->ev_status[k], hipEventDisableTiming));
    }
    NEK_HIP(hipHostMalloc((void **)&S->fin, MAX_SLOTS * sizeof(FinArea), hipHostMallocDefault));
    for (int i = MAX_SLOTS - 1; i >= 0; --i) S->free_index.push_back(i);
    nek_server *raw = S.get();
    for (int k = 0; k < PREP_THREADS; ++k) S->workers.emplace_back([raw] { raw->worker_loop(); });
    *out = S.release();
    return NEK_OK;
}

int nek_server_submit(nek_server *srv, const nek_request *req, uint64_t *id) {
    clear_error();
    if (!srv || !req || !req->b) return fail(NEK_ERR_ARG, "nek_server_submit: null argument");
    if (req->N < 1 || req->N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_server_submit: degree must be in 1..15");
    if (req->precision != NEK_PREC_F64 && !is_mixed(req->precision))
        return fail(NEK_ERR_UNSUPPORTED, "nek_server_submit: unknown precision");
    if (req->max_iter < 0) return fail(NEK_ERR_ARG, "nek_server_submit: max_iter must be >= 0");
    if (req->mem != NEK_MEM_HOST && req->mem != NEK_MEM_DEVICE)
        return fail(NEK_ERR_ARG, "nek_server_submit: mem must be NEK_MEM_HOST or NEK_MEM_DEVICE");
    const bool mesh = req->g != nullptr;
    const bool on_device = req->mem == NEK_MEM_DEVICE;
    int64_t E;
    if (mesh) {
        if (req->E < 1) return fail(NEK_ERR_ARG, "nek_server_submit: a mesh of the caller's needs E >= 1");
        if (!req->D || !req->glo) return fail(NEK_ERR_ARG, "nek_server_submit: a mesh of the caller's needs D, g and glo");
        E = req->E;
    } else {
        if (req->Ex < 1 || req->Ey < 1 || req->Ez < 1) return fail(NEK_ERR_ARG, "nek_server_submit: box sizes must be >= 1");
        E = (int64_t)req->Ex * req->Ey * req->Ez;
    }
    if (on_device && (!aligned8(req->b) || (mesh && (!aligned8(req->g) || !aligned8(req->D) || !aligned8(req->glo)))))
        return fail(NEK_ERR_ARG, "nek_server_submit: device arrays must be 8-byte aligned");
    if (E > ((int64_t)1 << 31)) return fail(NEK_ERR_ARG, "nek_server_submit: E*(N+1)^3 must be < 2^31");
    const int64_t P = E * n3_of(req->N);
    if (P >= ((int64_t)1 << 31)) return fail(NEK_ERR_ARG, "nek_server_submit: E*(N+1)^3 must be < 2^31");
    auto R = std::make_unique<Request>();
    R->id = srv->next_id++;
    R->spec = *req;   // the arrays are read later, not copied here
    R->mesh = mesh;
    R->on_device = on_device;
    R->E = E;
    R->P = P;
    R->fp = footprint_of(E, req->N, req->precision);
    if (R->fp.total > srv->budget)
        return fail(NEK_ERR_NOMEM, "nek_server_submit: the request alone exceeds the budget");
    R->t_submit = srv->clock();
    if (id) *id = R->id;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->prep_queue.push_back(R.get());
    }
    srv->cv.notify_one();
    srv->waiting.push_back(std::move(R));
    return NEK_OK;
}

int nek_server_step(nek_server *srv, int iters, int *active, int *queued) {
    clear_error();
    if (!srv) return fail(NEK_ERR_ARG, "nek_server_step: null server");
    return srv->step(iters, active, queued);
}

int nek_server_poll(nek_server *srv, nek_result *out, int max, int *n) {
    clear_error();
    if (!srv || !n || (max > 0 && !out)) return fail(NEK_ERR_ARG, "nek_server_poll: null argument");
    int k = 0;
    while (k < max && !srv->results.empty()) {
        out[k++] = srv->results.front();
        srv->results.pop_front();
    }
    *n = k;
    return NEK_OK;
}

int nek_server_fetch(nek_server *srv, uint64_t id, double *x_host) {
    clear_error();
    if (!srv || !x_host) return fail(NEK_ERR_ARG, "nek_server_fetch: null argument");
    auto it = srv->done.find(id);
    if (it == srv->done.end()) return fail(NEK_ERR_STATE, "nek_server_fetch: no finished solve with this id");
    Slot *S = it->second.get();
    NEK_HIP(hipMemcpyAsync(x_host, S->x, (size_t)S->req->P * sizeof(double), hipMemcpyDeviceToHost,
                           srv->copy_stream));
    NEK_HIP(hipStreamSynchronize(srv->copy_stream));
    (void)hipFreeAsync(S->x, srv->stream);
    srv->used -= S->req->fp.x;
    srv->done.erase(it);
    return NEK_OK;
}

double nek_server_clock(const nek_server *srv) { return srv ? srv->clock() : 0.0; }

int nek_server_destroy(nek_server *srv) {
    clear_error();
    if (!srv) return NEK_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    for (auto &t : srv->workers)
        if (t.joinable()) t.join();
    hipError_t e = hipStreamSynchronize(srv->stream);
    for (auto &s : srv->slots) {
        if (s->arena) (void)hipFree(s->arena);
        if (s->x) (void)hipFree(s->x);
        if (s->ev_upload) (void)hipEventDestroy(s->ev_upload);
        if (s->ev_fin) (void)hipEventDestroy(s->ev_fin);
    }
    for (auto &kv : srv->done)
        if (kv.second->x) (void)hipFree(kv.second->x);
    for (int k = 0; k < 2; ++k) {
        (void)hipHostFree(srv->tables[k].host);
        (void)hipFree(srv->tables[k].dev);
        (void)hipEventDestroy(srv->tables[k].ev);
        (void)hipFree(srv->status_dev[k]);
        (void)hipHostFree(srv->status_host[k]);
        (void)hipEventDestroy(srv->ev_status[k]);
    }
    (void)hipHostFree(srv->fin);
    srv->pinned.release_all();
    (void)hipStreamDestroy(srv->copy_stream);
    (void)hipStreamDestroy(srv->stream);
    delete srv;
    if (e != hipSuccess) return check_hip(e, "nek_server_destroy: hipStreamSynchronize");
    return NEK_OK;
}

}  // extern "C"
