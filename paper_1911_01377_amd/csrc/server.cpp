// Serving: continuous batching of independent periodic cells.
//
// A worker thread owns one HIP stream.  Each step advances every running
// request by one evaluation with one pass of the batched kernels (the same
// kernel bodies as a one-box evaluation, driven by a device table of the
// boxes in the batch), launched one by one or replayed from a captured HIP
// graph (option use_graph).  Between steps the
// worker retires finished requests (their outputs copied back through pinned
// staging) and admits waiting ones into free batch slots when their resident
// workspace fits in the device arena.
//
// Stream order carries every dependency: a newly admitted request's uploads
// (inputs, matrices, descriptor) are enqueued after the steps already in
// flight and before the step that first uses them; a finished request's
// outputs are copied after its last step; its slot and arena region are
// reused only after that copy has completed (its event).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "philox.h"
#include "useries_internal.h"

using namespace useries;

namespace {

constexpr size_t kAlign = 256;
constexpr int kRing = 4;          // pinned batch tables in rotation
constexpr int kMaxSkip = 64;      // admission rounds a waiting head lets later requests pass it

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator of byte ranges of the device arena.
class Arena {
public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

// Byte offsets of one request's resident device workspace.  It opens with
// what goes up at admission (charges, matrices, zeroed column counters,
// positions: one copy) followed by what comes down at the end (positions,
// forces, energies: one copy); the slot's pinned staging mirrors that prefix.
struct Layout {
    size_t q, mat[3], col_count, xyz, forces, energies, up_bytes, prefix, coord, sorted, perm,
        slots, cl_info, cl_col, cl_z, fnear, qpart, pair_parts, far_parts, qstats, col_start,
        col_fill, clus_start, bpre, zbin, rho, tgrid, phi, total;
};

Layout make_layout(const HostPlan& hp, int n, int n_evals) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align_up(std::max<size_t>(bytes, 1));
        return r;
    };
    const size_t c = (size_t)n;
    const size_t ncm = (size_t)hp.ncol_max;
    const size_t clmax = (size_t)pair_blocks(n, hp.ncol_max);
    const size_t ng = (size_t)hp.grid[0] * hp.grid[1] * hp.grid[2];
    L.q = take(4 * c);
    for (int a = 0; a < 3; ++a) L.mat[a] = take(hp.mats[a].size());
    L.col_count = take(4 * ncm);
    L.xyz = take(12 * c);
    L.up_bytes = L.xyz + 12 * c;
    L.forces = take(12 * c);
    L.energies = take(8 * (size_t)n_evals);
    L.prefix = L.energies + 8 * (size_t)n_evals;
    L.coord = take(16 * c);
    L.sorted = take(16 * c);
    L.perm = take(4 * c);
    L.slots = take(4 * c);
    L.cl_info = take(8 * clmax);
    L.cl_col = take(4 * clmax);
    L.cl_z = take(8 * clmax);
    L.fnear = take(16 * c);
    L.qpart = take(16 * ((c + 255) / 256));
    L.pair_parts = take(8 * clmax);
    L.far_parts = take(8 * (size_t)far_parts(hp.conv));
    L.qstats = take(16);
    L.col_start = take(4 * (ncm + 1));
    L.col_fill = take(4 * ncm);
    L.clus_start = take(4 * (ncm + 1));
    // two-launch binning's per-block column prefixes (the columns of n charges)
    const int ncol = hp.bin.nc[0] * hp.bin.nc[1];
    L.bpre = take(bin_local_ok(n, ncol) ? 4 * ((c + 255) / 256) * (size_t)(ncol + 1) : 0);
    L.zbin = take(4 * ncm * (size_t)(hp.grid[2] + 1));
    L.rho = take(4 * ng);
    L.tgrid = take(4 * ng * (size_t)hp.conv.nterms);
    L.phi = take(4 * ng);
    L.total = o;
    return L;
}

struct Req {
    uint64_t ticket = 0;
    useries_request r{};
    HostPlan hp;
    Layout lay{};
    int items[BK_COUNT] = {0};
    bool local = false;                      // two-launch binning
    size_t lds = 0, lds_z = 0, lds_g = 0;   // dynamic LDS of conv_xy, conv_z and gather
    int P = 0;                               // stencil half width
    // shared with API threads (under the server mutex)
    int state = USERIES_PENDING;
    int err_code = USERIES_OK;
    std::string err_msg;
    double t_submit = -1, t_admit = -1, t_done = -1;
    // worker only
    int slot = -1;
    size_t off = 0;
    int step = 0;
    int skipped = 0;
    hipEvent_t done_ev = nullptr;
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct useries_server_s {
    int device = 0;
    hipStream_t st = nullptr;
    int precision = USERIES_PLAIN_FP32;
    int max_slots = 1;
    useries_server_opts o{};
    useries_opts popts{};
    size_t budget = 0;
    char* arena_base = nullptr;
    Arena arena;
    // the batch table and the slots' box descriptors, uploaded together each
    // step from a ring of pinned copies: [table | max_slots descriptors]
    char* d_tabdesc = nullptr;
    BatchTable* d_table = nullptr;
    BoxDesc* d_desc = nullptr;
    BoxDesc* h_desc = nullptr;     // current descriptors (host) [max_slots]
    char* h_ring = nullptr;        // pinned [kRing][ring_stride]
    size_t ring_stride = 0;
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int ring_next = 0;
    struct Slot {
        Req* req = nullptr;
        char* staging = nullptr;
        size_t cap = 0;
    };
    std::vector<Slot> slots;
    std::vector<char*> old_staging;   // outgrown pinned buffers, freed at destruction (a free would
                                      // wait for the device)
    int grid[BK_COUNT] = {0};
    int lds_limit = 0;
    // by the dynamic LDS sizes and the stencil half width
    std::map<std::tuple<size_t, size_t, size_t, int, bool, int>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_objs;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    // shared state
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> incoming;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool held = false;       // admissions paused (useries_server_hold)
    bool broken = false;
    std::string broken_msg;
    int64_t stats[6] = {0};
    std::thread worker;

    // worker-only state
    std::deque<Req*> pending;
    std::vector<Req*> active;
    std::vector<Req*> finishing;
    std::deque<int> inflight;
    std::vector<hipEvent_t> ev_pool;

    hipEvent_t get_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    void set_state(Req* R, int state, int code = USERIES_OK, const std::string& msg = {}) {
        std::lock_guard<std::mutex> lk(mu);
        R->state = state;
        if (state == USERIES_RUNNING) R->t_admit = seconds_since(t0);
        if (state == USERIES_DONE || state == USERIES_ERROR) {
            R->t_done = seconds_since(t0);
            R->err_code = code;
            R->err_msg = msg;
            cv_done.notify_all();
        }
    }

    // the kernels of one step, in order, on the server stream
    // P: the stencil half width shared by the step's boxes, 0 if they differ;
    // exact: some box evaluates leading far terms as Gaussians in its near part;
    // bins: bit 0 some box bins in two launches, bit 1 some box in four
    hipError_t enqueue_kernels(size_t lds, size_t lds_z, size_t lds_g, int P, bool exact,
                               int bins) {
        const bool bf = precision == USERIES_BF16X3;
        hipError_t e;
        if ((bins & 1) && (e = launch_bin_local_batch(d_table, d_desc, grid[BK_BINLOCAL], st)))
            return e;
        if (bins & 2) {
            if ((e = launch_encode_batch(d_table, d_desc, grid[BK_ENCODE], st))) return e;
            if ((e = launch_scan_batch(d_table, d_desc, grid[BK_SCAN], st))) return e;
            if ((e = launch_scatter_batch(d_table, d_desc, grid[BK_SCATTER], st))) return e;
            if ((e = launch_colsort_batch(d_table, d_desc, grid[BK_COLSORT], st))) return e;
        }
        if ((bins & 1) && (e = launch_colbuild_batch(d_table, d_desc, grid[BK_COLBUILD], st)))
            return e;
        if ((e = launch_pair_batch(d_table, d_desc, popts.poly_degree, exact, grid[BK_PAIR], st))) return e;
        if ((e = launch_spread_batch(d_table, d_desc, P, grid[BK_SPREAD], st))) return e;
        if ((e = launch_conv_xy_batch(d_table, d_desc, bf, lds, grid[BK_CONV_XY], st))) return e;
        if ((e = launch_conv_z_batch(d_table, d_desc, bf, lds_z, grid[BK_CONV_Z], st))) return e;
        if ((e = launch_gather_batch(d_table, d_desc, P, lds_g, grid[BK_GATHER], st))) return e;
        return launch_displace_batch(d_table, d_desc, grid[BK_DISPLACE], st);
    }

    hipError_t graph_for(size_t lds, size_t lds_z, size_t lds_g, int P, bool exact, int bins,
                         hipGraphExec_t* out) {
        const std::tuple<size_t, size_t, size_t, int, bool, int> key(lds, lds_z, lds_g, P, exact,
                                                                     bins);
        auto it = graphs.find(key);
        if (it != graphs.end()) {
            *out = it->second;
            return hipSuccess;
        }
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e) return e;
        const hipError_t el = enqueue_kernels(lds, lds_z, lds_g, P, exact, bins);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(st, &g);
        if (el) {
            if (g) hipGraphDestroy(g);
            return el;
        }
        if (e) return e;
        hipGraphExec_t ex = nullptr;
        if ((e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0))) {
            hipGraphDestroy(g);
            return e;
        }
        graph_objs.push_back(g);
        graphs[key] = ex;
        {
            std::lock_guard<std::mutex> lk(mu);
            stats[5] += 1;
        }
        *out = ex;
        return hipSuccess;
    }

    // Put R on the device in slot s at arena offset off.
    hipError_t activate(Req* R, int s, size_t off) {
        Slot& S = slots[s];
        const HostPlan& hp = R->hp;
        const int n = (int)R->r.n;
        hipError_t e;
        const Layout& L = R->lay;
        if (S.cap < L.prefix) {
            if (S.staging) old_staging.push_back(S.staging);
            S.staging = nullptr;
            S.cap = 0;
            // pinned allocations take milliseconds: at least 2 MiB (a 60k-charge
            // box), twice the need beyond that
            const size_t want = std::max<size_t>(2 * L.prefix, (size_t)2 << 20);
            if ((e = hipHostMalloc((void**)&S.staging, want, hipHostMallocDefault))) return e;
            S.cap = want;
        }
        char* base = arena_base + off;
        char* stg = S.staging;
        BoxDesc& d = h_desc[s];
        std::memset(&d, 0, sizeof d);
        d.bin = hp.bin;
        d.pair = hp.pair;
        d.grid = hp.gridargs;
        d.conv = hp.conv;
        d.fin = hp.fin;
        d.ncol = hp.bin.nc[0] * hp.bin.nc[1];
        d.nq = (n + 255) / 256;
        d.npb = hp.fin.n_pair_parts;
        d.ngb = gather_blocks(hp.gridargs);
        d.n_evals = R->r.n_evals;
        d.disp_sigma = (float)R->r.disp_sigma;
        d.key[0] = (uint32_t)R->r.seed;
        d.key[1] = (uint32_t)(R->r.seed >> 32);
        d.xyz = (float*)(base + L.xyz);
        d.q = (const float*)(base + L.q);
        d.forces = (float*)(base + L.forces);
        d.energies = (double*)(base + L.energies);
        d.coord = (uint4*)(base + L.coord);
        d.sorted = (uint4*)(base + L.sorted);
        d.perm = (int*)(base + L.perm);
        d.slots = (int*)(base + L.slots);
        d.cl_col = (int*)(base + L.cl_col);
        d.cl_info = (int2*)(base + L.cl_info);
        d.cl_z = (uint2*)(base + L.cl_z);
        d.fnear = (float4*)(base + L.fnear);
        d.qpart = (double*)(base + L.qpart);
        d.pair_parts = (double*)(base + L.pair_parts);
        d.far_parts = (double*)(base + L.far_parts);
        d.qstats = (double*)(base + L.qstats);
        d.col_count = (int*)(base + L.col_count);
        d.col_start = (int*)(base + L.col_start);
        d.col_fill = (int*)(base + L.col_fill);
        d.clus_start = (int*)(base + L.clus_start);
        d.bpre = R->local ? (int*)(base + L.bpre) : nullptr;
        d.zbin = (int*)(base + L.zbin);
        d.rho = (float*)(base + L.rho);
        d.tgrid = (float*)(base + L.tgrid);
        d.phi = (float*)(base + L.phi);
        d.kx = (const float*)(base + L.mat[0]);
        d.ky = (const float*)(base + L.mat[1]);
        d.kz = (const float*)(base + L.mat[2]);

        // one upload: charges, matrices, zeroed column counters, positions (the
        // descriptor goes up with the next step's batch table)
        std::memcpy(stg + L.q, R->r.q, 4 * (size_t)n);
        for (int a = 0; a < 3; ++a)
            std::memcpy(stg + L.mat[a], hp.mats[a].data(), hp.mats[a].size());
        std::memset(stg + L.col_count, 0, 4 * (size_t)hp.ncol_max);
        std::memcpy(stg + L.xyz, R->r.xyz, 12 * (size_t)n);
        if ((e = hipMemcpyAsync(base, stg, L.up_bytes, hipMemcpyHostToDevice, st))) return e;
        R->slot = s;
        R->off = off;
        R->step = 0;
        S.req = R;
        for (int a = 0; a < 3; ++a) std::vector<uint8_t>().swap(R->hp.mats[a]);
        active.push_back(R);
        set_state(R, USERIES_RUNNING);
        return hipSuccess;
    }

    int free_slot() const {
        for (int s = 0; s < max_slots; ++s)
            if (!slots[s].req) return s;
        return -1;
    }

    hipError_t admit() {
        for (auto it = pending.begin(); it != pending.end();) {
            const int s = free_slot();
            if (s < 0) break;
            Req* R = *it;
            size_t off = 0;
            if (!arena.alloc(R->lay.total, &off)) {
                if (it == pending.begin() && ++R->skipped > kMaxSkip) break;
                ++it;
                continue;
            }
            const hipError_t e = activate(R, s, off);
            if (e) {
                arena.release(off, R->lay.total);
                return e;
            }
            it = pending.erase(it);
        }
        return hipSuccess;
    }

    hipError_t launch_step() {
        const int r = ring_next;
        ring_next = (ring_next + 1) % kRing;
        hipError_t e;
        if (ring_used[r] && (e = hipEventSynchronize(ring_ev[r]))) return e;
        char* ring = h_ring + (size_t)r * ring_stride;
        BatchTable& T = *reinterpret_cast<BatchTable*>(ring);
        const int nb = (int)active.size();
        T.nbox = nb;
        for (int k = 0; k < BK_COUNT; ++k) T.off[k][0] = 0;
        size_t lds = 0, lds_z = 0, lds_g = 0;
        int P = -1;
        bool exact = false;
        int bins = 0;
        for (int i = 0; i < nb; ++i) {
            Req* R = active[i];
            exact = exact || R->hp.near_exact > 0;
            bins |= R->local ? 1 : 2;
            T.slot[i] = R->slot;
            T.step[i] = R->step;
            for (int k = 0; k < BK_COUNT; ++k) {
                int items = R->items[k];
                if (k == BK_DISPLACE && !(R->step + 1 < R->r.n_evals && R->r.disp_sigma > 0))
                    items = 0;
                T.off[k][i + 1] = T.off[k][i] + items;
            }
            lds = std::max(lds, R->lds);
            lds_z = std::max(lds_z, R->lds_z);
            lds_g = std::max(lds_g, R->lds_g);
            P = (P < 0 || P == R->P) ? R->P : 0;
        }
        P = std::max(P, 0);
        std::memcpy(ring + align_up(sizeof(BatchTable)), h_desc, sizeof(BoxDesc) * max_slots);
        if ((e = hipMemcpyAsync(d_tabdesc, ring, ring_stride, hipMemcpyHostToDevice, st)))
            return e;
        if (o.use_graph) {
            hipGraphExec_t ex = nullptr;
            if ((e = graph_for(lds, lds_z, lds_g, P, exact, bins, &ex))) return e;
            if ((e = hipGraphLaunch(ex, st))) return e;
        } else if ((e = enqueue_kernels(lds, lds_z, lds_g, P, exact, bins))) {
            return e;
        }
        if ((e = hipEventRecord(ring_ev[r], st))) return e;
        ring_used[r] = true;
        inflight.push_back(r);
        {
            std::lock_guard<std::mutex> lk(mu);
            stats[0] += 1;
            stats[3] = std::max<int64_t>(stats[3], nb);
            stats[4] += nb;
        }
        // requests whose last evaluation this step was: copy their outputs back
        std::vector<Req*> still;
        still.reserve(active.size());
        for (Req* R : active) {
            R->step += 1;
            if (R->step < R->r.n_evals) {
                still.push_back(R);
                continue;
            }
            char* base = arena_base + R->off;
            char* stg = slots[R->slot].staging;
            const size_t n = (size_t)R->r.n;
            // one download: [positions,] forces, energies
            const size_t from = R->r.xyz_final ? R->lay.xyz : R->lay.forces;
            if ((e = hipMemcpyAsync(stg + from, base + from, R->lay.prefix - from,
                                    hipMemcpyDeviceToHost, st)))
                return e;
            R->done_ev = get_event();
            if (!R->done_ev) return hipErrorOutOfMemory;
            if ((e = hipEventRecord(R->done_ev, st))) return e;
            finishing.push_back(R);
        }
        active.swap(still);
        return hipSuccess;
    }

    // complete finished requests whose copies have landed
    hipError_t retire() {
        std::vector<Req*> left;
        for (Req* R : finishing) {
            const hipError_t q = hipEventQuery(R->done_ev);
            if (q == hipErrorNotReady) {
                left.push_back(R);
                continue;
            }
            if (q != hipSuccess) return q;
            const char* stg = slots[R->slot].staging;
            const size_t n = (size_t)R->r.n;
            std::memcpy(R->r.forces, stg + R->lay.forces, 12 * n);
            std::memcpy(R->r.energies, stg + R->lay.energies, 8 * (size_t)R->r.n_evals);
            if (R->r.xyz_final) std::memcpy(R->r.xyz_final, stg + R->lay.xyz, 12 * n);
            ev_pool.push_back(R->done_ev);
            R->done_ev = nullptr;
            arena.release(R->off, R->lay.total);
            slots[R->slot].req = nullptr;
            R->slot = -1;
            {
                std::lock_guard<std::mutex> lk(mu);
                stats[1] += R->r.n_evals;
                stats[2] += 1;
            }
            set_state(R, USERIES_DONE);
        }
        finishing.swap(left);
        return hipSuccess;
    }

    // a device error ends the server: every request not done fails
    void fail_all(hipError_t e, const char* where) {
        const std::string msg = std::string("serving ") + where + ": " + hipGetErrorString(e);
        {
            std::lock_guard<std::mutex> lk(mu);
            broken = true;
            broken_msg = msg;
            for (Req* R : incoming) pending.push_back(R);
            incoming.clear();
        }
        for (auto* list : {&active, &finishing}) {
            for (Req* R : *list) set_state(R, USERIES_ERROR, USERIES_EHIP, msg);
            list->clear();
        }
        for (Req* R : pending) set_state(R, USERIES_ERROR, USERIES_EHIP, msg);
        pending.clear();
        inflight.clear();
    }

    void run() {
        hipSetDevice(device);
        for (;;) {
            bool hold;
            {
                std::unique_lock<std::mutex> lk(mu);
                while (!incoming.empty()) {
                    pending.push_back(incoming.front());
                    incoming.pop_front();
                }
                hold = held && !stop;
                if (hold && active.empty() && finishing.empty() && inflight.empty()) {
                    cv_work.wait(lk, [&] { return stop || !held || !incoming.empty(); });
                    continue;
                }
                if (pending.empty() && active.empty() && finishing.empty()) {
                    if (stop) break;
                    if (inflight.empty()) {
                        cv_work.wait(lk, [&] { return stop || !incoming.empty(); });
                        continue;
                    }
                }
            }
            if (broken) {
                // drain: reject whatever arrives until destroyed
                for (Req* R : pending)
                    set_state(R, USERIES_ERROR, USERIES_EHIP, broken_msg);
                pending.clear();
                continue;
            }
            hipError_t e;
            if ((e = retire())) {
                fail_all(e, "retire");
                continue;
            }
            if (!hold && (e = admit())) {
                fail_all(e, "admit");
                continue;
            }
            if (!active.empty() && (int)inflight.size() < o.inflight) {
                if ((e = launch_step())) fail_all(e, "step");
                continue;
            }
            if (!inflight.empty()) {
                const int r = inflight.front();
                inflight.pop_front();
                if ((e = hipEventSynchronize(ring_ev[r]))) fail_all(e, "sync");
                continue;
            }
            if (!finishing.empty()) {
                if ((e = hipEventSynchronize(finishing.front()->done_ev))) fail_all(e, "sync");
                continue;
            }
            if (!hold && !pending.empty() && active.empty()) {
                // nothing on the device and the head does not fit an empty arena:
                // cannot happen for requests accepted by submit; fail it rather than spin
                Req* R = pending.front();
                pending.pop_front();
                set_state(R, USERIES_ERROR, USERIES_ENOMEM, "request does not fit the arena");
            }
        }
    }

    ~useries_server_s() {
        if (worker.joinable()) {
            {
                std::lock_guard<std::mutex> lk(mu);
                stop = true;
            }
            cv_work.notify_all();
            worker.join();
        }
        if (st) hipStreamSynchronize(st);
        for (auto& g : graphs) hipGraphExecDestroy(g.second);
        for (auto g : graph_objs) hipGraphDestroy(g);
        for (auto e : ev_pool) hipEventDestroy(e);
        for (auto e : ring_ev)
            if (e) hipEventDestroy(e);
        for (auto& s : slots)
            if (s.staging) hipHostFree(s.staging);
        for (char* b : old_staging) hipHostFree(b);
        delete[] h_desc;
        if (h_ring) hipHostFree(h_ring);
        hipFree(d_tabdesc);
        hipFree(arena_base);
        if (st) hipStreamDestroy(st);
    }
};

extern "C" {

int useries_server_default_opts(useries_server_opts* o) {
    if (!o) return set_last_error(USERIES_EINVAL, "NULL opts");
    o->construction = USERIES_C1;
    o->b = 2.0;
    o->nterms_tol = 1e-8;
    o->poly_degree = 0;
    o->use_graph = 0;
    o->inflight = 2;
    return USERIES_OK;
}

int useries_server_create(useries_server_t* out, size_t hbm_budget_bytes, int max_slots,
                          int precision, const useries_server_opts* opts) {
    if (!out) return set_last_error(USERIES_EINVAL, "NULL argument");
    *out = nullptr;
    if (max_slots < 1 || max_slots > kMaxBatch)
        return set_last_error(USERIES_EINVAL, "max_slots must lie in [1, 64]");
    if (precision != USERIES_PLAIN_FP32 && precision != USERIES_BF16X3)
        return set_last_error(USERIES_EINVAL, "unknown precision");
    if (hbm_budget_bytes < ((size_t)1 << 20))
        return set_last_error(USERIES_EINVAL, "hbm_budget_bytes below 1 MiB");
    useries_server_opts o;
    useries_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.inflight < 1 || o.inflight > 4) return set_last_error(USERIES_EINVAL, "inflight out of [1, 4]");
    if (o.poly_degree <= 0) o.poly_degree = precision == USERIES_BF16X3 ? 5 : 7;
    if (o.poly_degree < 4 || o.poly_degree > kMaxPolyDeg)
        return set_last_error(USERIES_EINVAL, "poly_degree out of [4, 14]");

    std::unique_ptr<useries_server_s> S(new useries_server_s());
    S->precision = precision;
    S->max_slots = max_slots;
    S->o = o;
    useries_default_opts(&S->popts);
    S->popts.construction = o.construction;
    S->popts.precision = precision;
    S->popts.nterms_tol = o.nterms_tol;
    S->popts.poly_degree = o.poly_degree;
    S->popts.spectral = 0;   // the batched convolutions take dense terms only
    S->budget = hbm_budget_bytes / kAlign * kAlign;
    hipError_t e;
    if ((e = hipGetDevice(&S->device))) return set_last_error(USERIES_EHIP, hipGetErrorString(e));
    int cu = 0;
    hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, S->device);
    hipDeviceGetAttribute(&S->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, S->device);
    cu = std::max(cu, 1);
    // persistent grids: a few resident blocks per compute unit for each kernel
    S->grid[BK_BINLOCAL] = 4 * cu;
    S->grid[BK_COLBUILD] = 2 * cu;
    S->grid[BK_ENCODE] = 4 * cu;
    S->grid[BK_SCAN] = max_slots;
    S->grid[BK_SCATTER] = 4 * cu;
    S->grid[BK_COLSORT] = 4 * cu;
    S->grid[BK_PAIR] = 16 * cu;
    S->grid[BK_SPREAD] = 2 * cu;
    S->grid[BK_CONV_XY] = 2 * cu;
    S->grid[BK_CONV_Z] = 4 * cu;
    S->grid[BK_GATHER] = 4 * cu;
    S->grid[BK_DISPLACE] = 2 * cu;
    S->ring_stride = align_up(sizeof(BatchTable)) + align_up(sizeof(BoxDesc) * max_slots);
    S->h_desc = new BoxDesc[max_slots]();
    if ((e = hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking)) ||
        (e = hipMalloc((void**)&S->d_tabdesc, S->ring_stride)) ||
        (e = hipHostMalloc((void**)&S->h_ring, S->ring_stride * kRing, hipHostMallocDefault)))
        return set_last_error(USERIES_EHIP, std::string("server setup: ") + hipGetErrorString(e));
    S->d_table = reinterpret_cast<BatchTable*>(S->d_tabdesc);
    S->d_desc = reinterpret_cast<BoxDesc*>(S->d_tabdesc + align_up(sizeof(BatchTable)));
    for (auto& ev : S->ring_ev)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)))
            return set_last_error(USERIES_EHIP, hipGetErrorString(e));
    if ((e = hipMalloc((void**)&S->arena_base, S->budget)))
        return set_last_error(USERIES_ENOMEM, std::string("arena: ") + hipGetErrorString(e));
    S->arena.reset(S->budget);
    S->slots.resize(max_slots);
    S->worker = std::thread([p = S.get()] { p->run(); });
    *out = S.release();
    return USERIES_OK;
}

int useries_submit(useries_server_t S, const useries_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket) return set_last_error(USERIES_EINVAL, "NULL argument");
    const useries_request& r = *req;
    if (r.n < 1 || r.n > INT_MAX / 4) return set_last_error(USERIES_EINVAL, "n out of range");
    if (!r.xyz || !r.q || !r.energies || !r.forces)
        return set_last_error(USERIES_EINVAL, "NULL buffer");
    if (r.n_evals < 1) return set_last_error(USERIES_EINVAL, "n_evals must be >= 1");
    if (!(r.disp_sigma >= 0) || !std::isfinite(r.disp_sigma))
        return set_last_error(USERIES_EINVAL, "disp_sigma must be finite and >= 0");
    std::unique_ptr<Req> R(new Req());
    R->r = r;
    std::string err;
    int rc = build_host_plan(&R->hp, r.box, r.r_c, S->o.b, 0.0, 0, r.grid, &S->popts, &err);
    if (rc) return set_last_error(rc, err);
    const int n = (int)r.n;
    choose_columns(&R->hp, n);
    const HostPlan& hp = R->hp;
    R->lds = conv_xy_lds_bytes(hp.conv);
    R->lds_z = conv_z_lds_bytes(hp.conv);
    R->lds_g = gather_lds_bytes(hp.P);
    R->P = hp.P;
    if (S->lds_limit > 0 && std::max({R->lds, R->lds_z, R->lds_g}) > (size_t)S->lds_limit)
        return set_last_error(USERIES_EINVAL, "grid and term count need more LDS than the device has");
    R->lay = make_layout(hp, n, r.n_evals);
    if (R->lay.total > S->budget)
        return set_last_error(USERIES_ENOMEM, "request workspace exceeds the server's budget");
    const int nq = (n + 255) / 256;
    const int kB = 8;   // spreading brick edge
    const int ncol = hp.bin.nc[0] * hp.bin.nc[1];
    R->local = bin_local_ok(n, ncol);
    if (R->local) {
        R->items[BK_BINLOCAL] = nq;
        R->items[BK_COLBUILD] = ncol;
    } else {
        R->items[BK_ENCODE] = nq;
        R->items[BK_SCAN] = 1;
        R->items[BK_SCATTER] = nq;
        R->items[BK_COLSORT] = ncol;
    }
    R->items[BK_PAIR] = hp.fin.n_pair_parts;
    R->items[BK_SPREAD] = ((hp.grid[0] + kB - 1) / kB) * ((hp.grid[1] + kB - 1) / kB) *
                          ((hp.grid[2] + kB - 1) / kB);
    R->items[BK_CONV_XY] = hp.grid[2] * hp.conv.nterms;
    R->items[BK_CONV_Z] = conv_z_blocks(hp.conv);
    R->items[BK_GATHER] = gather_blocks(hp.gridargs) + 1;   // the bricks, then the energy total
    R->items[BK_DISPLACE] = nq;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->broken) return set_last_error(USERIES_EHIP, S->broken_msg);
    if (S->stop) return set_last_error(USERIES_ESTATE, "server is shutting down");
    R->ticket = S->next_ticket++;
    R->t_submit = seconds_since(S->t0);
    *ticket = R->ticket;
    Req* raw = R.get();
    S->all.emplace(R->ticket, std::move(R));
    S->incoming.push_back(raw);
    S->cv_work.notify_one();
    return USERIES_OK;
}

int useries_server_hold(useries_server_t S, int hold) {
    if (!S) return set_last_error(USERIES_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->held = hold != 0;
    }
    S->cv_work.notify_all();
    return USERIES_OK;
}

int useries_poll(useries_server_t S, uint64_t ticket, int* state) {
    if (!S || !state) return set_last_error(USERIES_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_last_error(USERIES_ENOTFOUND, "unknown ticket");
    *state = it->second->state;
    if (*state == USERIES_ERROR) set_last_error(it->second->err_code, it->second->err_msg);
    return USERIES_OK;
}

int useries_wait(useries_server_t S, uint64_t ticket, int* state) {
    if (!S || !state) return set_last_error(USERIES_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_last_error(USERIES_ENOTFOUND, "unknown ticket");
    Req* R = it->second.get();
    S->cv_done.wait(lk, [&] { return R->state == USERIES_DONE || R->state == USERIES_ERROR; });
    *state = R->state;
    if (*state == USERIES_ERROR) set_last_error(R->err_code, R->err_msg);
    return USERIES_OK;
}

int useries_request_times(useries_server_t S, uint64_t ticket, double* t_submit, double* t_admit,
                          double* t_done) {
    if (!S) return set_last_error(USERIES_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_last_error(USERIES_ENOTFOUND, "unknown ticket");
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_admit) *t_admit = it->second->t_admit;
    if (t_done) *t_done = it->second->t_done;
    return USERIES_OK;
}

int useries_server_stats(useries_server_t S, int64_t out[6]) {
    if (!S || !out) return set_last_error(USERIES_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    for (int k = 0; k < 6; ++k) out[k] = S->stats[k];
    return USERIES_OK;
}

int useries_server_destroy(useries_server_t S) {
    if (!S) return set_last_error(USERIES_EINVAL, "NULL server");
    delete S;
    return USERIES_OK;
}

void useries_philox4x32_10(const uint32_t counter[4], const uint32_t key[2], uint32_t out[4]) {
    Philox4 c;
    for (int k = 0; k < 4; ++k) c.v[k] = counter[k];
    const Philox4 r = philox4x32_10(c, key[0], key[1]);
    for (int k = 0; k < 4; ++k) out[k] = r.v[k];
}

}  // extern "C"
