// server.hip -- serving loop for assembly jobs and page-op jobs: admission by a
// device-memory budget and a slot limit, resident connectivity and CSR structures keyed by
// topology and built without stopping the scheduler, one fused numeric launch per
// (dimension, precision, rows-per-block) class and one batch-plan launch per precision for
// the page-op jobs in every scheduler tick.
//
// The scheduler thread owns every HIP call of the server (one compute stream plus one
// stream for structure builds).  Public calls only touch host state under the server mutex.
// Job lifecycle:
//   pending --admit--> waiting for its structure (assembly jobs whose structure is being
//   built; the build is polled every tick) --ready--> in flight (inputs copied, compute
//   launched, copy-back queued) --compute event--> finished (latency taken) --copy event-->
//   done (memory freed)
#include "internal.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace pf;

namespace {

constexpr int RING = 4;  // job-table staging buffers in flight

struct Topo {
    uint64_t key = 0;
    int dim = 0;
    int64_t nn = 0, ne = 0;
    int32_t* d_elems = nullptr;
    pf_csr* csr = nullptr;
    size_t bytes = 0;  // accounted device bytes (estimate until built)
    int refs = 0;
    uint64_t last_use = 0;
    enum { NEW, BUILDING, BUILT, FAILED } state = NEW;
    pf_status status = PF_OK;  // of a failed build
    bool cached = false;
};

struct TickEvents {
    hipEvent_t num = nullptr, copy = nullptr;
    ~TickEvents() {
        if (num) (void)hipEventDestroy(num);
        if (copy) (void)hipEventDestroy(copy);
    }
};

struct SJob {
    uint64_t ticket = 0;
    pf_job spec{};
    pf_job_result res{};
    Topo* topo = nullptr;
    // assembly jobs: counters, coordinates, K and M values, parts of one allocation d_mem
    double* d_coords = nullptr;
    void* d_valsK = nullptr;
    void* d_valsM = nullptr;
    int64_t* d_ctr = nullptr;
    void* d_mem = nullptr;
    void* d_pg = nullptr;  // page-op jobs: A, B, inv(A), A*B and det(A) in one allocation
    int slot = -1;  // row of the pinned counter block
    size_t bytes = 0;
    int stage = 0;  // 0 pending, 1 waiting or in flight, 2 compute done, 3 done
    std::shared_ptr<TickEvents> ev;
};

size_t elem_bytes(int32_t prec) { return prec == PF_F32 ? 4 : 8; }
bool is_pages(const pf_job& j) { return j.kind == PF_JOB_PAGES; }

// upper bound of the nonzeros before the structure is built
int64_t nnz_bound(const pf_job& j) {
    const int64_t nlb = j.dim + 1;
    return std::min<int64_t>(j.ne * nlb * nlb, j.nn * 64);
}

// device bytes a structure may hold while it is built (its largest moment: the connectivity,
// the resident arrays and the build's scratch); once built it holds csr_bytes
size_t topo_estimate(const pf_job& j) {
    if (is_pages(j)) return 0;
    const int64_t m = j.ne * (j.dim + 1);
    return static_cast<size_t>(4 * m)                        // elems (released when the build ends)
           + static_cast<size_t>(8 * m + 12 * (j.nn + 1))     // compact adjacency, slot words, offsets, diagonal
           + static_cast<size_t>(4 * nnz_bound(j))            // col_idx
           + static_cast<size_t>(520 * (j.nn + 64))           // scratch: padded adjacency, row-pattern columns
           + static_cast<size_t>(j.nn / 256) + 4096;
}

// the device arrays of a page-op job, in one allocation: A, then B, inv(A), A*B (each
// count n^2 values, present when the ops need them), then det(A); offsets in values
struct PageLayout {
    int64_t a, b, x, c, det, total;
};
PageLayout page_layout(const pf_job& j) {
    const int64_t pg = j.count * j.order * j.order;
    PageLayout L{};
    int64_t o = 0;
    L.a = o;
    o += pg;
    L.b = (j.ops & PF_OP_MTIMES) ? o : -1;
    o += (j.ops & PF_OP_MTIMES) ? pg : 0;
    L.x = (j.ops & PF_OP_INV) ? o : -1;
    o += (j.ops & PF_OP_INV) ? pg : 0;
    L.c = (j.ops & PF_OP_MTIMES) ? o : -1;
    o += (j.ops & PF_OP_MTIMES) ? pg : 0;
    L.det = (j.ops & PF_OP_INV) ? o : -1;
    o += (j.ops & PF_OP_INV) ? j.count : 0;
    L.total = o;
    return L;
}

size_t job_estimate(const pf_job& j, int64_t nnz) {
    if (is_pages(j)) return static_cast<size_t>(page_layout(j).total) * elem_bytes(j.prec) + 256;
    return static_cast<size_t>(j.nn * j.dim * 8) + 2 * static_cast<size_t>(nnz) * elem_bytes(j.prec) + 1280;
}

}  // namespace

struct pf_server {
    size_t budget = 0;
    int max_slots = 0;
    int flags = 0;
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SJob*> pending;
    std::vector<SJob*> waiting;  // admitted assembly jobs whose structure is being built
    std::vector<SJob*> active;
    std::unordered_map<uint64_t, std::unique_ptr<SJob>> jobs;
    std::map<uint64_t, Topo*> cache;
    uint64_t next_ticket = 1, use_clock = 0;
    int64_t unfinished = 0;  // submitted and not done (pending, being admitted, or in flight)
    bool stop = false;

    size_t used = 0, high = 0;
    pf_stats st{};
    std::vector<double> lat;

    hipStream_t s = nullptr, sbuild = nullptr;
    NumericJob* h_tab[RING] = {};
    NumericJob* d_tab[RING] = {};
    hipEvent_t tab_ev[RING] = {};
    bool tab_used[RING] = {};
    int ring = 0;
    pf_plan* plans[2][RING] = {};  // page-op jobs: per precision, a ring of batch plans
    int pring[2] = {0, 0};
    int64_t* h_ctr = nullptr;  // pinned, 4 per slot
    std::vector<int> free_slots;
    std::thread th;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void account(pf_server* S, long long delta) {
    S->used = static_cast<size_t>(static_cast<long long>(S->used) + delta);
    S->high = std::max(S->high, S->used);
}

// a structure's memory goes back to the pool in the order of the serving stream, which
// every use of it was enqueued on (its build, on the build stream, has ended): nothing waits
void destroy_topo(pf_server* S, Topo* t) {
    if (t->csr) csr_release(t->csr, S->s);
    if (t->d_elems) (void)hipFreeAsync(t->d_elems, S->s);
    account(S, -static_cast<long long>(t->bytes));
    delete t;
}

// evict resident structures nobody uses, least recently used first, until `need` fits
void make_room(pf_server* S, size_t need) {
    while (S->used + need > S->budget) {
        Topo* victim = nullptr;
        for (auto& kv : S->cache)
            if (kv.second->refs == 0 && (!victim || kv.second->last_use < victim->last_use)) victim = kv.second;
        if (!victim) return;
        S->cache.erase(victim->key);
        const auto t0 = std::chrono::steady_clock::now();
        destroy_topo(S, victim);
        S->st.evict_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        ++S->st.evictions;
    }
}

// structure of a job: resident (cache hit), or new (estimate accounted; built later).
// `cacheable` says whether a new structure may enter the cache under the job's key.
Topo* topo_for(pf_server* S, SJob* j, size_t& extra, bool& cacheable) {
    extra = 0;
    cacheable = j->spec.topology != 0 && !(S->flags & PF_SERVER_NOCACHE);
    if (cacheable) {
        auto it = S->cache.find(j->spec.topology);
        if (it != S->cache.end()) {
            if (it->second->dim == j->spec.dim && it->second->nn == j->spec.nn && it->second->ne == j->spec.ne)
                return it->second;
            cacheable = false;  // the key names another mesh: this job gets a private structure
        }
    }
    extra = topo_estimate(j->spec);
    return nullptr;
}

// start the build of a job's structure on the build stream (connectivity copied in, the
// symbolic phase enqueued); its end is found by poll_build
pf_status start_build(pf_server* S, SJob* j, Topo* t) {
    const pf_job& q = j->spec;
    const size_t eb = static_cast<size_t>(q.ne * (q.dim + 1)) * 4;
    t->state = Topo::BUILDING;
    PF_HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&t->d_elems), std::max<size_t>(eb, 16), S->sbuild));
    PF_HIP_TRY(hipMemcpyAsync(t->d_elems, q.elems, eb, hipMemcpyHostToDevice, S->sbuild));
    pf_status st = pf_csr_create(&t->csr);
    if (st != PF_OK) return st;
    return csr_symbolic_enqueue(t->csr, q.dim, q.nn, q.ne, t->d_elems, S->sbuild);
}

// a building structure whose status has reached the host becomes BUILT (exact bytes
// accounted) or FAILED; returns whether its state changed
bool poll_build(pf_server* S, Topo* t) {
    if (t->state != Topo::BUILDING) return false;
    pf_status st;
    if (!csr_symbolic_poll(t->csr, &st)) return false;
    std::lock_guard<std::mutex> lk(S->mu);
    if (t->d_elems) {  // the numeric phase reads only the structure and the coordinates
        (void)hipFreeAsync(t->d_elems, S->sbuild);
        t->d_elems = nullptr;
    }
    if (st == PF_OK) {
        const size_t exact = csr_bytes(t->csr);
        account(S, static_cast<long long>(exact) - static_cast<long long>(t->bytes));
        t->bytes = exact;
        t->state = Topo::BUILT;
    } else {
        t->state = Topo::FAILED;
        t->status = st;
        if (t->cached) {  // a failed build never serves another job
            S->cache.erase(t->key);
            t->cached = false;
        }
    }
    return true;
}

void finish(pf_server* S, SJob* j, pf_status status) {
    // caller holds the lock
    j->res.status = status;
    j->res.done = 1;
    j->stage = 3;
    --S->unfinished;
    if (status == PF_OK) {
        ++S->st.completed;
        if (is_pages(j->spec)) S->st.pages += j->spec.count;
        else S->st.elements += j->spec.ne;
        S->lat.push_back(j->res.finished - j->res.arrival);
        if (S->st.completed == 1 || j->res.arrival < S->st.first_arrival) S->st.first_arrival = j->res.arrival;
        S->st.last_finish = std::max(S->st.last_finish, j->res.finished);
    } else {
        ++S->st.failed;
    }
}

// release a job's device memory (stream-ordered) and its structure reference
void release(pf_server* S, SJob* j) {
    for (void** p : {&j->d_mem, &j->d_pg}) {
        if (*p) (void)hipFreeAsync(*p, S->s);
        *p = nullptr;
    }
    j->d_coords = nullptr;
    j->d_valsK = j->d_valsM = nullptr;
    j->d_ctr = nullptr;
    account(S, -static_cast<long long>(j->bytes));
    j->bytes = 0;
    if (j->slot >= 0) S->free_slots.push_back(j->slot);
    j->slot = -1;
    if (Topo* t = j->topo) {
        --t->refs;
        if (!t->cached && t->refs == 0) {
            // a structure still building is destroyed once its build has ended
            if (t->state == Topo::BUILDING) (void)hipStreamSynchronize(S->sbuild);
            destroy_topo(S, t);
        }
        j->topo = nullptr;
    }
}

// Stage 1 of a tick, under the lock: move admissible pending jobs into `batch`.
void admit(pf_server* S, std::vector<SJob*>& batch) {
    const double t = S->now();
    while (!S->pending.empty() &&
           static_cast<int>(S->active.size() + S->waiting.size() + batch.size()) < S->max_slots) {
        SJob* j = S->pending.front();
        if (j->res.arrival > t) break;  // not arrived yet (a pre-submitted trace)
        size_t extra = 0;
        bool cacheable = false;
        Topo* hit = is_pages(j->spec) ? nullptr : topo_for(S, j, extra, cacheable);
        const int64_t nnz = (hit && hit->state == Topo::BUILT) ? csr_nnz(hit->csr) : nnz_bound(j->spec);
        const size_t need = job_estimate(j->spec, nnz) + extra;
        if (S->used + need > S->budget) make_room(S, need);
        if (S->used + need > S->budget) {  // head of the queue waits for memory
            ++S->st.admit_waits;
            break;
        }
        S->pending.pop_front();
        if (hit) {
            j->topo = hit;
            ++S->st.cache_hits;
        } else if (!is_pages(j->spec)) {
            Topo* tp = new Topo();
            tp->key = j->spec.topology;
            tp->dim = j->spec.dim;
            tp->nn = j->spec.nn;
            tp->ne = j->spec.ne;
            tp->bytes = extra;
            tp->cached = cacheable;
            account(S, static_cast<long long>(extra));
            if (tp->cached) S->cache[tp->key] = tp;
            j->topo = tp;
            ++S->st.cache_misses;
        }
        if (j->topo) {
            j->topo->refs++;
            j->topo->last_use = ++S->use_clock;
        }
        j->bytes = job_estimate(j->spec, nnz);
        account(S, static_cast<long long>(j->bytes));
        j->slot = S->free_slots.back();
        S->free_slots.pop_back();
        j->res.admitted = t;
        j->stage = 1;
        batch.push_back(j);
    }
}

struct TickCounts {
    int64_t launches = 0, launched = 0;
};

// inputs of a ready assembly job (values sized by its structure), or the error
pf_status assembly_inputs(pf_server* S, SJob* j) {
    const pf_job& q = j->spec;
    const int64_t nnz = csr_nnz(j->topo->csr);
    if ((q.valsK || q.valsM) && nnz > q.vals_cap) return fail(PF_ELIMIT, "pf_server: vals_cap below nnz");
    const size_t es = elem_bytes(q.prec);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        const size_t exact = job_estimate(q, nnz);
        account(S, static_cast<long long>(exact) - static_cast<long long>(j->bytes));
        j->bytes = exact;
        j->res.nnz = nnz;
    }
    // one stream-ordered allocation (its release, like any, costs the scheduler a runtime call)
    auto part = [](size_t b) { return (std::max<size_t>(b, 16) + 255) & ~size_t(255); };
    const size_t b_ctr = part(32), b_xyz = part(q.nn * q.dim * 8), b_val = part(nnz * es);
    hipError_t e = hipMallocAsync(&j->d_mem, b_ctr + b_xyz + 2 * b_val, S->s);
    if (e == hipSuccess) {
        char* base = static_cast<char*>(j->d_mem);
        j->d_ctr = reinterpret_cast<int64_t*>(base);
        j->d_coords = reinterpret_cast<double*>(base + b_ctr);
        j->d_valsK = base + b_ctr + b_xyz;
        j->d_valsM = base + b_ctr + b_xyz + b_val;
        e = hipMemcpyAsync(j->d_coords, q.coords, q.nn * q.dim * 8, hipMemcpyHostToDevice, S->s);
    }
    if (e == hipSuccess) e = hipMemsetAsync(j->d_ctr, 0, 32, S->s);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? PF_ENOMEM : PF_EHIP,
                    std::string("pf_server: job inputs: ") + hipGetErrorString(e));
    return PF_OK;
}

// inputs of a page-op job: one device allocation, pages A (and B) copied in
pf_status page_inputs(pf_server* S, SJob* j) {
    const pf_job& q = j->spec;
    const PageLayout L = page_layout(q);
    const size_t es = elem_bytes(q.prec);
    const size_t pg = static_cast<size_t>(q.count * q.order * q.order) * es;
    hipError_t e = hipMallocAsync(&j->d_pg, static_cast<size_t>(L.total) * es, S->s);
    char* base = static_cast<char*>(j->d_pg);
    if (e == hipSuccess) e = hipMemcpyAsync(base + L.a * es, q.a, pg, hipMemcpyHostToDevice, S->s);
    if (e == hipSuccess && L.b >= 0) e = hipMemcpyAsync(base + L.b * es, q.b, pg, hipMemcpyHostToDevice, S->s);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? PF_ENOMEM : PF_EHIP,
                    std::string("pf_server: page inputs: ") + hipGetErrorString(e));
    j->res.nnz = 0;
    j->res.routed = -1;
    return PF_OK;
}

// Stage 2 of a tick, without the lock: inputs of the ready jobs, fused compute launches,
// copies back.  Jobs that fail go to `failed` with their status.
void run_tick(pf_server* S, std::vector<SJob*>& ready, std::vector<std::pair<SJob*, pf_status>>& failed,
              TickCounts& tc) {
    std::vector<SJob*> ok, pages;
    for (SJob* j : ready) {
        const pf_status st = is_pages(j->spec) ? page_inputs(S, j) : assembly_inputs(S, j);
        if (st != PF_OK) failed.emplace_back(j, st);
        else if (is_pages(j->spec)) pages.push_back(j);
        else ok.push_back(j);
    }
    if (ok.empty() && pages.empty()) return;
    auto ev = std::make_shared<TickEvents>();
    (void)hipEventCreateWithFlags(&ev->num, hipEventDisableTiming);
    (void)hipEventCreateWithFlags(&ev->copy, hipEventDisableTiming);
    std::vector<SJob*> launched;
    if (S->flags & PF_SERVER_NOFUSE) {
        for (SJob* j : ok) {
            pf_status st = pf_assemble(j->topo->csr, static_cast<pf_dtype>(j->spec.prec), j->d_coords, nullptr,
                                       nullptr, nullptr, j->d_valsK, j->d_valsM, &j->spec.fb, j->d_ctr, S->s);
            if (st == PF_OK) {
                launched.push_back(j);
                ++tc.launches;
            } else {
                failed.emplace_back(j, st);
            }
        }
    } else if (!ok.empty()) {
        // group by class, fill the ring's staging table, one copy, one launch per class
        const int r = S->ring;
        S->ring = (S->ring + 1) % RING;
        if (S->tab_used[r]) (void)hipEventSynchronize(S->tab_ev[r]);
        std::map<std::tuple<int, int, int>, std::vector<SJob*>> cls;
        for (SJob* j : ok) {
            const pf_dtype pr = static_cast<pf_dtype>(j->spec.prec);
            if (csr_nn(j->topo->csr) == 0) {
                launched.push_back(j);
                continue;
            }
            cls[{j->spec.dim, static_cast<int>(pr), numeric_class(j->topo->csr, pr)}].push_back(j);
        }
        int n = 0;
        struct Launch {
            int dim, prec, nr, first, count, wmax;
            int64_t blocks;
        };
        std::vector<Launch> ls;
        for (auto& kv : cls) {
            Launch L{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), n, 0, 0, 0};
            for (SJob* j : kv.second) {
                const pf_dtype pr = static_cast<pf_dtype>(j->spec.prec);
                numeric_describe(j->topo->csr, j->d_coords, j->d_valsK, j->d_valsM, &j->spec.fb, j->d_ctr, L.blocks,
                                 &S->h_tab[r][n]);
                L.blocks += numeric_blocks(j->topo->csr, pr);
                L.wmax = std::max(L.wmax, numeric_wmax(j->topo->csr, L.nr));
                ++n;
                ++L.count;
            }
            ls.push_back(L);
        }
        hipError_t e = hipMemcpyAsync(S->d_tab[r], S->h_tab[r], sizeof(NumericJob) * n, hipMemcpyHostToDevice, S->s);
        (void)hipEventRecord(S->tab_ev[r], S->s);
        S->tab_used[r] = true;
        for (const Launch& L : ls) {
            pf_status st = e == hipSuccess ? numeric_launch_many(L.dim, static_cast<pf_dtype>(L.prec), L.nr,
                                                                 S->d_tab[r] + L.first, L.count, L.blocks, L.wmax, S->s)
                                           : fail(PF_EHIP, std::string("pf_server: job table: ") + hipGetErrorString(e));
            for (auto& kv : cls)
                if (std::get<0>(kv.first) == L.dim && std::get<1>(kv.first) == L.prec && std::get<2>(kv.first) == L.nr)
                    for (SJob* j : kv.second) {
                        // the job's long rows (rare), which the fused launch skips
                        pf_status sj = st;
                        if (sj == PF_OK)
                            sj = numeric_long(j->topo->csr, static_cast<pf_dtype>(L.prec), j->d_coords, j->d_valsK,
                                              j->d_valsM, &j->spec.fb, j->d_ctr, S->s);
                        if (sj == PF_OK) launched.push_back(j);
                        else failed.emplace_back(j, sj);
                    }
            ++tc.launches;
        }
    }
    // page-op jobs: one batch-plan launch per precision (its graph replayed), or one plan
    // launch per job without fusion
    for (int pi = 0; pi < 2 && !pages.empty(); ++pi) {
        const pf_dtype pr = pi == 0 ? PF_F32 : PF_F64;
        std::vector<SJob*> js;
        for (SJob* j : pages)
            if (j->spec.prec == pr) js.push_back(j);
        const size_t nfuse = (S->flags & PF_SERVER_NOFUSE) ? 1 : js.size();
        for (size_t k0 = 0; k0 < js.size(); k0 += nfuse) {
            const size_t k1 = std::min(js.size(), k0 + nfuse);
            pf_plan*& plan = S->plans[pi][S->pring[pi]];
            S->pring[pi] = (S->pring[pi] + 1) % RING;
            pf_status st = plan ? PF_OK : pf_plan_create(pr, S->max_slots, nullptr, &plan);
            std::vector<pf_group> gs;
            for (size_t k = k0; k < k1; ++k) {
                SJob* j = js[k];
                const PageLayout L = page_layout(j->spec);
                char* base = static_cast<char*>(j->d_pg);
                const size_t es = elem_bytes(pr);
                pf_group g{};
                g.order = j->spec.order;
                g.ops = j->spec.ops;
                g.count = j->spec.count;
                g.a = base + L.a * es;
                g.b = L.b >= 0 ? base + L.b * es : nullptr;
                g.x = L.x >= 0 ? base + L.x * es : nullptr;
                g.c = L.c >= 0 ? base + L.c * es : nullptr;
                g.det = L.det >= 0 ? base + L.det * es : nullptr;
                gs.push_back(g);
            }
            if (st == PF_OK) st = pf_plan_set_groups(plan, gs.data(), static_cast<int32_t>(gs.size()));
            if (st == PF_OK) st = pf_plan_run(plan, nullptr, S->s);
            for (size_t k = k0; k < k1; ++k) {
                if (st == PF_OK) launched.push_back(js[k]);
                else failed.emplace_back(js[k], st);
            }
            ++tc.launches;
        }
    }
    (void)hipEventRecord(ev->num, S->s);
    for (SJob* j : launched) {
        const pf_job& q = j->spec;
        const size_t es = elem_bytes(q.prec);
        if (is_pages(q)) {
            const PageLayout L = page_layout(q);
            const char* base = static_cast<const char*>(j->d_pg);
            const size_t pg = static_cast<size_t>(q.count * q.order * q.order) * es;
            if (q.x && L.x >= 0) (void)hipMemcpyAsync(q.x, base + L.x * es, pg, hipMemcpyDeviceToHost, S->s);
            if (q.c && L.c >= 0) (void)hipMemcpyAsync(q.c, base + L.c * es, pg, hipMemcpyDeviceToHost, S->s);
            if (q.det && L.det >= 0)
                (void)hipMemcpyAsync(q.det, base + L.det * es, q.count * es, hipMemcpyDeviceToHost, S->s);
        } else {
            const size_t bytes = static_cast<size_t>(j->res.nnz) * es;
            if (q.valsK && bytes) (void)hipMemcpyAsync(q.valsK, j->d_valsK, bytes, hipMemcpyDeviceToHost, S->s);
            if (q.valsM && bytes) (void)hipMemcpyAsync(q.valsM, j->d_valsM, bytes, hipMemcpyDeviceToHost, S->s);
            (void)hipMemcpyAsync(S->h_ctr + 4 * j->slot, j->d_ctr, 32, hipMemcpyDeviceToHost, S->s);
        }
        j->ev = ev;
    }
    (void)hipEventRecord(ev->copy, S->s);
    tc.launched = static_cast<int64_t>(launched.size());
}

void loop(pf_server* S) {
    (void)hipSetDevice(S->device);
    std::vector<SJob*> batch, ready, still;
    std::vector<std::pair<SJob*, pf_status>> failed;
    for (;;) {
        batch.clear();
        ready.clear();
        failed.clear();
        bool progress = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && S->unfinished == 0) break;
            if (S->pending.empty() && S->active.empty() && S->waiting.empty()) {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            admit(S, batch);
        }
        // newly admitted jobs: page jobs and jobs with a built structure are ready now; a
        // new structure starts building (at most one build per structure)
        for (SJob* j : batch) {
            if (is_pages(j->spec)) {
                ready.push_back(j);
                continue;
            }
            Topo* t = j->topo;
            if (t->state == Topo::NEW) {
                const auto b0 = std::chrono::steady_clock::now();
                const pf_status st = start_build(S, j, t);
                S->st.build_start_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - b0).count();
                if (st != PF_OK) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    t->state = Topo::FAILED;
                    t->status = st;
                    if (t->cached) {
                        S->cache.erase(t->key);
                        t->cached = false;
                    }
                }
            }
            if (t->state == Topo::BUILT) ready.push_back(j);
            else if (t->state == Topo::FAILED) failed.emplace_back(j, t->status);
            else S->waiting.push_back(j);
        }
        // structures whose build has ended release their waiting jobs
        still.clear();
        for (SJob* j : S->waiting) {
            Topo* t = j->topo;
            if (poll_build(S, t)) progress = true;
            if (t->state == Topo::BUILT) ready.push_back(j);
            else if (t->state == Topo::FAILED) failed.emplace_back(j, t->status);
            else still.push_back(j);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->waiting.swap(still);
        }
        if (!ready.empty()) {
            TickCounts tc;
            const auto k0 = std::chrono::steady_clock::now();
            run_tick(S, ready, failed, tc);
            const double dk = std::chrono::duration<double>(std::chrono::steady_clock::now() - k0).count();
            progress = true;
            std::lock_guard<std::mutex> lk(S->mu);
            S->st.tick_s += dk;
            for (SJob* j : ready) S->active.push_back(j);
            ++S->st.ticks;
            S->st.launches += tc.launches;
            S->st.max_batch = std::max(S->st.max_batch, tc.launched);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto& f : failed) {
                SJob* j = f.first;
                S->active.erase(std::remove(S->active.begin(), S->active.end(), j), S->active.end());
                j->res.finished = j->res.copied = S->now();
                release(S, j);
                finish(S, j, f.second);
                progress = true;
            }
            const double t = S->now();
            for (size_t i = 0; i < S->active.size();) {
                SJob* j = S->active[i];
                if (j->stage == 1 && j->ev && hipEventQuery(j->ev->num) == hipSuccess) {
                    j->res.finished = t;
                    j->stage = 2;
                    progress = true;
                }
                if (j->stage == 2 && hipEventQuery(j->ev->copy) == hipSuccess) {
                    j->res.copied = S->now();
                    if (!is_pages(j->spec)) j->res.routed = S->h_ctr[4 * j->slot];
                    release(S, j);
                    finish(S, j, PF_OK);
                    j->ev.reset();
                    S->active[i] = S->active.back();
                    S->active.pop_back();
                    progress = true;
                    continue;
                }
                ++i;
            }
            if (progress) S->cv_done.notify_all();
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

pf_status check_job(const pf_job* q) {
    if (!q) return fail(PF_EINVAL, "pf_server_submit: job is NULL");
    if (q->prec != PF_F32 && q->prec != PF_F64) return fail(PF_EDTYPE, "pf_server_submit: prec");
    if (q->kind == PF_JOB_PAGES) {
        if (q->order < 1 || q->order > 4) return fail(PF_EORDER, "pf_server_submit: page order must be 1..4");
        if (q->ops <= 0 || (q->ops & ~(PF_OP_INV | PF_OP_MTIMES)))
            return fail(PF_EINVAL, "pf_server_submit: page ops must be PF_OP_INV and/or PF_OP_MTIMES");
        if (q->count <= 0 || !q->a || ((q->ops & PF_OP_MTIMES) && !q->b))
            return fail(PF_EINVAL, "pf_server_submit: empty page job or NULL host pages");
        if (q->count >= (int64_t(1) << 40)) return fail(PF_ELIMIT, "pf_server_submit: too many pages");
        return PF_OK;
    }
    if (q->kind != PF_JOB_ASSEMBLY) return fail(PF_EINVAL, "pf_server_submit: unknown job kind");
    if (q->dim != 2 && q->dim != 3) return fail(PF_EORDER, "pf_server_submit: dim must be 2 or 3");
    if (q->nn <= 0 || q->ne <= 0 || !q->coords || !q->elems)
        return fail(PF_EINVAL, "pf_server_submit: empty mesh or NULL host arrays");
    if (q->vals_cap < 0) return fail(PF_EINVAL, "pf_server_submit: negative vals_cap");
    if (q->nn >= INT32_MAX || q->ne * (q->dim + 1) >= INT32_MAX)
        return fail(PF_ELIMIT, "pf_server_submit: mesh too large for 32-bit indices");
    return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_server_create(size_t hbm_budget, int32_t max_slots, int32_t flags, pf_server** out) {
    if (!out) return fail(PF_EINVAL, "pf_server_create: out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 65536) return fail(PF_EINVAL, "pf_server_create: max_slots must be 1..65536");
    if (hbm_budget == 0) return fail(PF_EINVAL, "pf_server_create: zero budget");
    if (flags & ~(PF_SERVER_NOFUSE | PF_SERVER_NOCACHE)) return fail(PF_EINVAL, "pf_server_create: flags");
    pf_server* S = new (std::nothrow) pf_server();
    if (!S) return fail(PF_ENOMEM, "pf_server_create: host allocation");
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    S->flags = flags;
    S->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->sbuild, hipStreamNonBlocking);
    for (int r = 0; r < RING && e == hipSuccess; ++r) {
        e = hipHostMalloc(reinterpret_cast<void**>(&S->h_tab[r]), sizeof(NumericJob) * max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->d_tab[r]), sizeof(NumericJob) * max_slots);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->tab_ev[r], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S->h_ctr), 32 * static_cast<size_t>(max_slots),
                                           hipHostMallocDefault);
    if (e != hipSuccess) {
        pf_server_destroy(S);
        return fail(PF_EHIP, std::string("pf_server_create: ") + hipGetErrorString(e));
    }
    for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
    try {
        S->th = std::thread(loop, S);
    } catch (...) {
        pf_server_destroy(S);
        return fail(PF_ENOMEM, "pf_server_create: cannot start the scheduler thread");
    }
    *out = S;
    return PF_OK;
}

double pf_server_now(const pf_server* S) { return S ? S->now() : 0.0; }

pf_status pf_server_submit(pf_server* S, const pf_job* q, uint64_t* ticket) {
    if (!S) return fail(PF_EINVAL, "pf_server_submit: server is NULL");
    pf_status st = check_job(q);
    if (st != PF_OK) return st;
    size_t need = 0;
    pf_server_footprint(q, &need);
    if (need > S->budget) return fail(PF_EBUDGET, "pf_server_submit: the job can never fit the memory budget");
    auto j = std::make_unique<SJob>();
    j->spec = *q;
    j->res.arrival = q->arrival < 0 ? S->now() : q->arrival;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(PF_ESTATE, "pf_server_submit: server is shutting down");
    j->ticket = S->next_ticket++;
    if (ticket) *ticket = j->ticket;
    S->pending.push_back(j.get());
    S->jobs[j->ticket] = std::move(j);
    ++S->st.submitted;
    ++S->unfinished;
    S->cv_work.notify_one();
    return PF_OK;
}

pf_status pf_server_footprint(const pf_job* q, size_t* bytes) {
    pf_status st = check_job(q);
    if (st != PF_OK) return st;
    if (!bytes) return fail(PF_EINVAL, "pf_server_footprint: bytes is NULL");
    *bytes = job_estimate(*q, nnz_bound(*q)) + topo_estimate(*q);
    return PF_OK;
}

pf_status pf_server_poll(pf_server* S, uint64_t ticket, pf_job_result* out) {
    if (!S) return fail(PF_EINVAL, "pf_server_poll: server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(PF_EINVAL, "pf_server_poll: unknown ticket");
    if (out) *out = it->second->res;
    return PF_OK;
}

pf_status pf_server_wait(pf_server* S, uint64_t ticket, pf_job_result* out) {
    if (!S) return fail(PF_EINVAL, "pf_server_wait: server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(PF_EINVAL, "pf_server_wait: unknown ticket");
    SJob* j = it->second.get();
    S->cv_done.wait(lk, [&] { return j->res.done != 0; });
    if (out) *out = j->res;
    return PF_OK;
}

pf_status pf_server_drain(pf_server* S) {
    if (!S) return fail(PF_EINVAL, "pf_server_drain: server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->unfinished == 0; });
    return PF_OK;
}

pf_status pf_server_stats(pf_server* S, pf_stats* out) {
    if (!S || !out) return fail(PF_EINVAL, "pf_server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    std::vector<double> l = S->lat;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
        if (l.empty()) return 0.0;
        const size_t k = std::min(l.size() - 1, static_cast<size_t>(p * (l.size() - 1) + 0.5));
        return l[k];
    };
    out->latency_p50 = pct(0.50);
    out->latency_p99 = pct(0.99);
    out->latency_max = l.empty() ? 0.0 : l.back();
    double sum = 0;
    for (double x : l) sum += x;
    out->latency_mean = l.empty() ? 0.0 : sum / l.size();
    const double span = out->last_finish - out->first_arrival;
    out->jobs_per_s = span > 0 ? out->completed / span : 0.0;
    out->elements_per_s = span > 0 ? out->elements / span : 0.0;
    out->pages_per_s = span > 0 ? out->pages / span : 0.0;
    out->hbm_in_use = static_cast<int64_t>(S->used);
    out->hbm_high_water = static_cast<int64_t>(S->high);
    return PF_OK;
}

void pf_server_destroy(pf_server* S) {
    if (!S) return;
    if (S->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        S->th.join();
    }
    if (S->s) (void)hipStreamSynchronize(S->s);
    for (auto& kv : S->cache) destroy_topo(S, kv.second);
    S->cache.clear();
    if (S->s) (void)hipStreamSynchronize(S->s);
    csr_pool_trim();
    for (auto& ring : S->plans)
        for (pf_plan* p : ring)
            if (p) pf_plan_destroy(p);
    for (int r = 0; r < RING; ++r) {
        if (S->h_tab[r]) (void)hipHostFree(S->h_tab[r]);
        if (S->d_tab[r]) (void)hipFree(S->d_tab[r]);
        if (S->tab_ev[r]) (void)hipEventDestroy(S->tab_ev[r]);
    }
    if (S->h_ctr) (void)hipHostFree(S->h_ctr);
    if (S->sbuild) (void)hipStreamDestroy(S->sbuild);
    if (S->s) (void)hipStreamDestroy(S->s);
    delete S;
}

}  // extern "C"
