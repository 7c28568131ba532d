// submit.hip -- batched submissions with tickets, and the cost-model dry run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <string>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <vector>

#include "devplan.hpp"
#include "plan.hpp"
#include "runtime.hpp"

using namespace spmm;

#define SPMM_TRY_HIP(call, what)                          \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_error(e_, what); \
    } while (0)

namespace {
// A ticket's completion event and the plans its work uses.  The table holds
// one reference; spmm_wait holds another while it waits, so the event stays
// valid even when a concurrent spmm_poll retires the ticket meanwhile.
struct Ticket {
    hipEvent_t done = nullptr;
    std::vector<spmm_plan_t *> plans;
    Ticket() = default;
    Ticket(const Ticket &) = delete;
    Ticket &operator=(const Ticket &) = delete;
    ~Ticket() {
        if (done) (void)hipEventDestroy(done);
    }
};
std::mutex g_tk_mu;
std::map<spmm_ticket, std::shared_ptr<Ticket>> g_tickets;
std::atomic<uint64_t> g_next_ticket{1};

// Under g_tk_mu: the ticket's plans are released exactly once, by whichever
// call takes it out of the table.
void retire(std::map<spmm_ticket, std::shared_ptr<Ticket>>::iterator it) {
    for (auto *p : it->second->plans) p->busy.fetch_sub(1);
    it->second->plans.clear();
    g_tickets.erase(it);
}
}  // namespace

// ------------------------------------------------------------------------------------------
// Batched submission: one descriptor table per kernel variant, copied from a
// pinned staging ring, executed by a captured graph of three persistent
// kernels (segment partials, then vector items, then windows).

namespace {

constexpr unsigned kBatchSegPerCu = 3;

struct VariantGraph {
    void *dtab = nullptr;  // BatchHeader (padded to 256 B) followed by entries
    size_t dcap = 0;
    hipGraphExec_t exec = nullptr;
    BatchGrids grids;
};

struct BatchCtx {
    hipStream_t capture = nullptr;
    std::map<uint64_t, VariantGraph> variants;
    static constexpr int kSlots = 4;
    void *pinned[kSlots] = {};
    size_t pinned_cap[kSlots] = {};
    hipEvent_t pinned_ev[kSlots] = {};
    int next = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

std::mutex g_batch_mu;
std::map<std::pair<int, hipStream_t>, BatchCtx> g_batch;

constexpr size_t kHeaderBytes = 256;
static_assert(sizeof(BatchHeader) <= kHeaderBytes, "batch header grew");

spmm_status ensure_device(void **p, size_t *cap, size_t bytes) {
    if (*cap >= bytes) return SPMM_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    size_t want = std::max(bytes, (size_t)1 << 16);
    hipError_t e = hipMalloc(p, want);
    if (e != hipSuccess) {
        *p = nullptr;
        return set_error(SPMM_ERR_OOM, std::string("hipMalloc(batch): ") + hipGetErrorString(e));
    }
    *cap = want;
    return SPMM_OK;
}

}  // namespace

extern "C" spmm_status spmm_submit(const spmm_work *items, int32_t count, void *stream,
                                   spmm_ticket *out) {
    if (!out || count < 0 || (count > 0 && !items)) return set_error(SPMM_ERR_INVALID, "bad arguments");
    *out = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int32_t i = 0; i < count; ++i) {
        spmm_status st = check_run(items[i].plan, items[i].B, items[i].ldb, items[i].C, items[i].ldc);
        if (st != SPMM_OK) return st;
    }
    int dev = 0;
    SPMM_TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
    int ncu = 0;
    SPMM_TRY_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
                 "hipDeviceGetAttribute");

    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchCtx &ctx = g_batch[{dev, s}];

    // run arguments, workspace layout and variant grouping
    std::vector<RunArgs> args(count);
    std::map<uint64_t, std::vector<int32_t>> groups;
    size_t ws_floats = 0;
    for (int32_t i = 0; i < count; ++i) {
        const spmm_plan_t *p = items[i].plan;
        if (p->hp.m == 0) continue;
        make_run_args(p, items[i].B, items[i].ldb, items[i].C, items[i].ldc, args[i]);
        // the batched window kernels stage 128-column panels
        set_window_panels(args[i], (int)p->hp.n, chunk_elems(p->hp.b_type), 128);
        ws_floats += workspace_floats(p->hp, true);
        const int E = args[i].vec_ok ? chunk_elems(p->hp.b_type) : 1;
        const int chunks = args[i].vec_ok ? args[i].np / E : args[i].np;
        const int cpl = chunks > 64 ? 2 : 1;
        const uint64_t key = (uint64_t)p->hp.val_type | ((uint64_t)p->hp.b_type << 4) |
                             ((uint64_t)p->hp.tile_type << 8) | ((uint64_t)args[i].vec_ok << 12) |
                             ((uint64_t)cpl << 16) | ((uint64_t)args[i].pipeline << 20);
        groups[key].push_back(i);
    }
    if (ws_floats * sizeof(float) > ctx.ws_bytes) {
        if (ctx.ws) {
            SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(batch workspace)");
            (void)hipFree(ctx.ws);
            ctx.ws = nullptr;
            ctx.ws_bytes = 0;
        }
        spmm_status st = ensure_device(&ctx.ws, &ctx.ws_bytes, ws_floats * sizeof(float));
        if (st != SPMM_OK) return st;
    }
    {
        size_t off = 0;
        for (int32_t i = 0; i < count; ++i) {
            const spmm_plan_t *p = items[i].plan;
            if (p->hp.m == 0) continue;
            args[i].work = static_cast<float *>(ctx.ws) + off;
            off += workspace_floats(p->hp, true);
        }
    }

    for (auto &kv : groups) {
        const uint64_t key = kv.first;
        const std::vector<int32_t> &idx = kv.second;
        const int32_t vt = key & 0xF, bt = (key >> 4) & 0xF, tt = (key >> 8) & 0xF;
        const int vec_ok = (key >> 12) & 0xF, cpl = (key >> 16) & 0xF, var = (key >> 20) & 0xF;
        // Work of each matrix (~ entries * N plus rows * N).  Whole matrices go
        // to the 8 XCDs by longest processing time, so that each XCD's L2
        // serves one matrix's B at a time.  While that leaves an XCD above 120%
        // of an even share, the largest matrix still placed whole is instead
        // cut into 8 contiguous chunks of its items of every kind, one per XCD
        // (a batch of a few matrices ends with all of them cut, so no XCD
        // idles), and the others are placed again.  Longest processing time
        // keeps every XCD below the even share plus the largest whole cost, so
        // no more than the matrices above 2.5% of the total are ever cut.
        std::vector<int32_t> order(idx.size());
        for (size_t j = 0; j < idx.size(); ++j) order[j] = (int32_t)j;
        auto cost = [&](int32_t j) {
            const spmm_plan_t *p = items[idx[j]].plan;
            return ((double)p->hp.nnz + (double)p->hp.m) * (double)p->hp.n;
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
        std::vector<int32_t> xcd_of(idx.size(), 0);
        std::vector<uint8_t> split(idx.size(), 0);
        double total = 0;
        for (int32_t j : order) total += cost(j);
        for (size_t ns = 0; ns <= order.size(); ++ns) {  // the ns largest are cut
            double load[8], share = 0;
            for (size_t t = 0; t < ns; ++t) share += cost(order[t]) / 8.0;
            for (int x = 0; x < 8; ++x) load[x] = share;
            for (size_t t = ns; t < order.size(); ++t) {
                int best = 0;
                for (int x = 1; x < 8; ++x)
                    if (load[x] < load[best]) best = x;
                xcd_of[order[t]] = best;
                load[best] += cost(order[t]);
            }
            if (*std::max_element(load, load + 8) <= 1.2 * total / 8.0 || ns == order.size()) {
                for (size_t t = 0; t < ns; ++t) split[order[t]] = 1;
                break;
            }
        }
        struct Ent {
            int32_t j;
            int64_t base[4], cnt[4];
        };
        std::vector<Ent> ents;
        int32_t x_first[9];
        for (int x = 0; x < 8; ++x) {
            x_first[x] = (int32_t)ents.size();
            for (int32_t j : order) {
                const spmm_plan_t *p = items[idx[j]].plan;
                const RunArgs &a = args[idx[j]];
                const int64_t n4[4] = {(int64_t)p->dp.n_seg * a.n_panels,
                                       (int64_t)p->dp.n_vitems * a.n_panels,
                                       (int64_t)p->dp.n_win * a.win_panels,
                                       (int64_t)p->dp.n_wpart * a.win_panels};
                Ent e{j, {0, 0, 0, 0}, {0, 0, 0, 0}};
                if (!split[j]) {
                    if (xcd_of[j] != x) continue;
                    for (int q = 0; q < 4; ++q) e.cnt[q] = n4[q];
                } else {
                    for (int q = 0; q < 4; ++q) {
                        e.base[q] = n4[q] * x / 8;
                        e.cnt[q] = n4[q] * (x + 1) / 8 - e.base[q];
                    }
                }
                ents.push_back(e);
            }
        }
        x_first[8] = (int32_t)ents.size();
        // host table
        const size_t bytes = kHeaderBytes + std::max<size_t>(ents.size(), 1) * sizeof(BatchEntry);
        BatchCtx &c = ctx;
        const int slot = c.next;
        c.next = (c.next + 1) % BatchCtx::kSlots;
        if (c.pinned_ev[slot]) SPMM_TRY_HIP(hipEventSynchronize(c.pinned_ev[slot]), "hipEventSynchronize(staging)");
        if (c.pinned_cap[slot] < bytes) {
            if (c.pinned[slot]) (void)hipHostFree(c.pinned[slot]);
            c.pinned[slot] = nullptr;
            c.pinned_cap[slot] = 0;
            size_t want = std::max(bytes, (size_t)1 << 16);
            hipError_t e = hipHostMalloc(&c.pinned[slot], want, hipHostMallocDefault);
            if (e != hipSuccess) return set_error(SPMM_ERR_OOM, "hipHostMalloc(batch table)");
            c.pinned_cap[slot] = want;
        }
        if (!c.pinned_ev[slot])
            SPMM_TRY_HIP(hipEventCreateWithFlags(&c.pinned_ev[slot], hipEventDisableTiming), "hipEventCreate");
        auto *hdr = static_cast<BatchHeader *>(c.pinned[slot]);
        auto *tab = reinterpret_cast<BatchEntry *>(static_cast<uint8_t *>(c.pinned[slot]) + kHeaderBytes);
        int64_t ns = 0, nv = 0, nw = 0, np_ = 0;
        for (int x = 0; x <= 8; ++x) hdr->x_entry[x] = x_first[x];
        for (size_t jj = 0; jj < ents.size(); ++jj) {
            const Ent &en = ents[jj];
            for (int x = 0; x < 8; ++x)
                if (x_first[x] == (int32_t)jj) {
                    hdr->x_seg[x] = (int32_t)ns;
                    hdr->x_vec[x] = (int32_t)nv;
                    hdr->x_win[x] = (int32_t)nw;
                    hdr->x_wpart[x] = (int32_t)np_;
                }
            const spmm_plan_t *p = items[idx[en.j]].plan;
            BatchEntry &e = tab[jj];
            e.P = p->dp;
            e.a = args[idx[en.j]];
            ns += en.cnt[0];
            nv += en.cnt[1];
            nw += en.cnt[2];
            np_ += en.cnt[3];
            if (ns > INT32_MAX || nv > INT32_MAX || nw > INT32_MAX || np_ > INT32_MAX)
                return set_error(SPMM_ERR_UNSUPPORTED, "batch has more than 2^31 items");
            e.seg_end = (int32_t)ns;
            e.vec_end = (int32_t)nv;
            e.win_end = (int32_t)nw;
            e.wpart_end = (int32_t)np_;
            e.seg_base = (int32_t)en.base[0];
            e.vec_base = (int32_t)en.base[1];
            e.win_base = (int32_t)en.base[2];
            e.wpart_base = (int32_t)en.base[3];
        }
        // XCDs with no entry start where the next one does
        for (int x = 7; x >= 0; --x)
            if (hdr->x_entry[x] == hdr->x_entry[x + 1]) {
                hdr->x_seg[x] = x < 7 ? hdr->x_seg[x + 1] : (int32_t)ns;
                hdr->x_vec[x] = x < 7 ? hdr->x_vec[x + 1] : (int32_t)nv;
                hdr->x_win[x] = x < 7 ? hdr->x_win[x + 1] : (int32_t)nw;
                hdr->x_wpart[x] = x < 7 ? hdr->x_wpart[x + 1] : (int32_t)np_;
            }
        hdr->x_seg[8] = (int32_t)ns;
        hdr->x_vec[8] = (int32_t)nv;
        hdr->x_win[8] = (int32_t)nw;
        hdr->x_wpart[8] = (int32_t)np_;
        hdr->count = (int32_t)ents.size();
        hdr->total_seg = (int32_t)ns;
        hdr->total_vec = (int32_t)nv;
        hdr->total_win = (int32_t)nw;
        hdr->total_wpart = (int32_t)np_;

        VariantGraph &vg = ctx.variants[key];
        if (vg.dcap < bytes) {
            if (vg.exec) {
                SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(batch table)");
                (void)hipGraphExecDestroy(vg.exec);
                vg.exec = nullptr;
            }
            spmm_status st = ensure_device(&vg.dtab, &vg.dcap, bytes);
            if (st != SPMM_OK) return st;
        }
        if (!vg.exec) {
            BatchGrids occ;
            SPMM_TRY_HIP(batch_occupancy(vt, bt, tt, vec_ok, cpl, var, &occ), "occupancy");
            // each kernel's grid is its resident workgroups per CU times the CUs,
            // in a multiple of 8 so that every XCD gets the same number; the
            // segment kernel takes at most 3 per CU, its fastest measured grid
            // (512 uneven f16 matrices: 1.72 / 1.40 / 1.43 / 1.56 / 1.64 ms at
            // 2 / 3 / 4 / 5 / 8 per CU, where it had shared the vector kernel's
            // 5; the vector kernel at 4 per CU, or at 6 with fewer registers,
            // was slower than at its own 5)
            auto fill = [&](unsigned per_cu) { return std::max(8u, (std::max(1u, per_cu) * (unsigned)ncu) & ~7u); };
            vg.grids.seg = fill(std::min(occ.seg, kBatchSegPerCu));
            vg.grids.vec = fill(occ.vec);
            vg.grids.win = fill(occ.win);
            if (!ctx.capture)
                SPMM_TRY_HIP(hipStreamCreateWithFlags(&ctx.capture, hipStreamNonBlocking), "hipStreamCreate");
            const auto *dh = static_cast<const BatchHeader *>(vg.dtab);
            const auto *dt = reinterpret_cast<const BatchEntry *>(static_cast<uint8_t *>(vg.dtab) + kHeaderBytes);
            SPMM_TRY_HIP(hipStreamBeginCapture(ctx.capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            hipError_t le = launch_batch(dh, dt, vt, bt, tt, vec_ok, cpl, var, vg.grids, ctx.capture);
            hipGraph_t graph = nullptr;
            hipError_t ce = hipStreamEndCapture(ctx.capture, &graph);
            if (le != hipSuccess) return hip_error(le, "batched launch (capture)");
            if (ce != hipSuccess) return hip_error(ce, "hipStreamEndCapture");
            hipError_t ie = hipGraphInstantiate(&vg.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                vg.exec = nullptr;
                return hip_error(ie, "hipGraphInstantiate");
            }
        }
        SPMM_TRY_HIP(hipMemcpyAsync(vg.dtab, c.pinned[slot], bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync(batch table)");
        SPMM_TRY_HIP(hipEventRecord(c.pinned_ev[slot], s), "hipEventRecord");
        SPMM_TRY_HIP(hipGraphLaunch(vg.exec, s), "hipGraphLaunch");
    }

    auto t = std::make_shared<Ticket>();
    hipError_t e = hipEventCreateWithFlags(&t->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        t->done = nullptr;
        return hip_error(e, "hipEventCreate");
    }
    e = hipEventRecord(t->done, s);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord");
    for (int32_t i = 0; i < count; ++i) {
        auto *p = const_cast<spmm_plan_t *>(items[i].plan);
        p->busy.fetch_add(1);
        t->plans.push_back(p);
    }
    const spmm_ticket id = g_next_ticket.fetch_add(1);
    std::lock_guard<std::mutex> lk2(g_tk_mu);
    g_tickets[id] = std::move(t);
    *out = id;
    return SPMM_OK;
}

extern "C" spmm_status spmm_poll(spmm_ticket id, int32_t *done) {
    if (!done) return set_error(SPMM_ERR_INVALID, "done is null");
    std::lock_guard<std::mutex> lk(g_tk_mu);
    auto it = g_tickets.find(id);
    if (it == g_tickets.end()) {  // unknown or already retired
        *done = 1;
        return SPMM_OK;
    }
    hipError_t e = hipEventQuery(it->second->done);
    if (e == hipErrorNotReady) {
        *done = 0;
        return SPMM_OK;
    }
    if (e != hipSuccess) return hip_error(e, "hipEventQuery");
    retire(it);
    *done = 1;
    return SPMM_OK;
}

extern "C" spmm_status spmm_wait(spmm_ticket id) {
    std::shared_ptr<Ticket> t;  // keeps the event alive while this call waits
    {
        std::lock_guard<std::mutex> lk(g_tk_mu);
        auto it = g_tickets.find(id);
        if (it == g_tickets.end()) return SPMM_OK;
        t = it->second;
    }
    hipError_t e = hipEventSynchronize(t->done);
    if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
    std::lock_guard<std::mutex> lk(g_tk_mu);
    auto it = g_tickets.find(id);
    if (it != g_tickets.end()) retire(it);
    return SPMM_OK;
}

// ------------------------------------------------------------------------------------------
// Dry run (Sec. 5.2.1): time the vector path on a uniformly random matrix and
// the MFMA path on fully dense 16-row windows, with the same N and B type.

namespace {
struct DeviceBuffer {
    void *p = nullptr;
    ~DeviceBuffer() {
        if (p) (void)hipFree(p);
    }
};

spmm_status time_plan(const spmm_csr &A, int32_t n, int32_t bt, const spmm_opts &o,
                      hipStream_t s, double *ms_per_run) {
    spmm_plan_t *p = nullptr;
    spmm_status st = spmm_plan(&A, n, bt, SPMM_F32, &o, &p);
    if (st != SPMM_OK) return st;
    std::unique_ptr<spmm_plan_t, spmm_status (*)(spmm_plan_t *)> guard(p, spmm_plan_destroy);
    const size_t sb = dtype_size(bt);
    DeviceBuffer B, C;
    if (hipMalloc(&B.p, (size_t)A.k * n * sb) != hipSuccess ||
        hipMalloc(&C.p, (size_t)A.m * n * 4) != hipSuccess)
        return set_error(SPMM_ERR_OOM, "dry run buffers");
    if (hipMemsetAsync(B.p, 0, (size_t)A.k * n * sb, s) != hipSuccess)
        return set_error(SPMM_ERR_DEVICE, "dry run memset");
    for (int w = 0; w < 2; ++w) {
        st = spmm_run(p, B.p, n, C.p, n, s);
        if (st != SPMM_OK) return st;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(SPMM_ERR_DEVICE, "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(SPMM_ERR_DEVICE, "event");
    }
    const int reps = 5;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == SPMM_OK; ++r) st = spmm_run(p, B.p, n, C.p, n, s);
    (void)hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SPMM_OK) return st;
    if (e != hipSuccess) return hip_error(e, "dry run sync");
    *ms_per_run = ms / reps;
    return SPMM_OK;
}
}  // namespace

extern "C" spmm_status spmm_dryrun(int32_t n, int32_t b_type, void *stream, double *p_vec,
                                   double *p_mfma) {
    if (n < 1 || !p_vec || !p_mfma || b_type < 0 || b_type > 2)
        return set_error(SPMM_ERR_INVALID, "bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t vt = b_type == SPMM_F32 ? SPMM_F32 : b_type;
    const int sv = dtype_size(vt);
    std::mt19937_64 rng(12345);

    // vector path: 2^18 rows, 16 uniformly random columns each
    {
        const int64_t m = 1 << 18, per = 16;
        std::vector<int64_t> rp(m + 1);
        std::vector<int32_t> ci(m * per);
        std::vector<uint8_t> v(m * per * sv, 0);
        for (int64_t r = 0; r <= m; ++r) rp[r] = r * per;
        for (auto &c : ci) c = (int32_t)(rng() % m);
        spmm_csr A{m, m, m * per, rp.data(), ci.data(), v.data(), vt, 0};
        spmm_opts o;
        spmm_opts_default(&o);
        o.mode = SPMM_MODE_PLAIN_F32;
        double ms = 0;
        spmm_status st = time_plan(A, n, b_type, o, s, &ms);
        if (st != SPMM_OK) return st;
        *p_vec = (double)A.nnz * n / (ms * 1e-3);
    }
    // matrix path: 2^14 windows of 16 rows, each a fully dense 16 x 64 block
    {
        const int64_t m = 1 << 18, per = 64;
        std::vector<int64_t> rp(m + 1);
        std::vector<int32_t> ci(m * per);
        std::vector<uint8_t> v(m * per * sv, 0);
        for (int64_t r = 0; r <= m; ++r) rp[r] = r * per;
        for (int64_t w = 0; w < m / 16; ++w) {
            std::vector<int32_t> cols(per);
            for (auto &c : cols) c = (int32_t)(rng() % m);
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            while ((int64_t)cols.size() < per) cols.push_back((cols.back() + 1) % m);
            for (int r = 0; r < 16; ++r)
                std::copy(cols.begin(), cols.end(), ci.begin() + (w * 16 + r) * per);
        }
        spmm_csr A{m, m, m * per, rp.data(), ci.data(), v.data(), vt, 0};
        spmm_opts o;
        spmm_opts_default(&o);
        o.mode = SPMM_MODE_MFMA_ONLY;
        o.window_h = 16;
        o.row_order = SPMM_ORDER_ORIGINAL_RANGES;
        double ms = 0;
        spmm_status st = time_plan(A, n, b_type, o, s, &ms);
        if (st != SPMM_OK) return st;
        *p_mfma = (double)A.nnz * n / (ms * 1e-3);  // every entry is a tile slot
    }
    return SPMM_OK;
}
