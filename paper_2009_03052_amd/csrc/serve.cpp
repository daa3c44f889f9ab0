// Serving: resident tables and a request loop. Requests are admitted against a
// device-memory budget (their outputs live in one pre-allocated arena), and the
// samples of every admitted request are interleaved into steps, each one launch
// of the serving sampler (plus the classifier for requests that ask for
// classes). A request that arrives while others run joins at the next step.
// AGS sessions run the rounds of adaptive graphlet sampling (Sec. 4.1) as
// requests: a round starts when the previous round of its session has finished,
// with the shape the session's controller picked from the earlier rounds.
//
// Every sample is fixed by its table, shape and (seed, stream, index), so a
// request gives the same rows alone as in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ags.hpp"
#include "arena.hpp"
#include "sampler.hpp"

namespace {

struct Request {
    int64_t id = 0;
    scc_request q{};
    int k = 0, shape = -1;
    uint64_t seed = 0, stream = 0, first = 0;
    int64_t bytes = 0, off = -1;
    int32_t *verts = nullptr;
    int8_t *par = nullptr;
    uint32_t *cls = nullptr;
    int64_t assigned = 0, done = 0;
    int status = SCC_OK;
    bool admitted = false, finished = false;
    double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
};

struct Session {
    int table = 0;
    uint64_t seed = 0, stream = 0;
    AgsState st;
    std::deque<int64_t> rounds;      // admitted rounds waiting for their turn
    bool busy = false;
    uint64_t next_first = 0;
    unsigned long long *dhist = nullptr;
    std::vector<unsigned long long> hh;
};

constexpr int STEP_BUFS = 2;

struct StepBuf {
    hipStream_t stream = nullptr;    // the step buffers alternate between two streams
    SampleArgs *hargs = nullptr, *dargs = nullptr;
    ServeClassArgs *hcls = nullptr, *dcls = nullptr;
    ServeChunk *hch = nullptr, *dch = nullptr;
    int64_t *hend = nullptr, *dend = nullptr;
    int *herr = nullptr, *derr = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<int64_t> req;        // request of each chunk
    int nch = 0;
    int64_t total = 0;
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct scc_server {
    std::vector<scc_table *> tables;
    scc_server_opts o{};
    hipStream_t st = nullptr, st2 = nullptr, side = nullptr;
    bool own_stream = false;
    DevMem mem;
    uint8_t *arena_base = nullptr;
    Arena arena;
    std::vector<std::vector<SampleArgs>> base;     // [table][shape + 1]
    std::vector<const uint16_t *> lut;
    std::vector<int> nclass;
    StepBuf sb[STEP_BUFS];
    int max_active = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Request> reqs;
    std::vector<int64_t> active;
    size_t rr = 0;
    std::deque<Session> sessions;     // a deque: opening a session moves no other
    int64_t next_id = 1;
    bool stop = false;
    int fatal = SCC_OK;
    std::thread th;
    std::chrono::steady_clock::time_point t0;
    // statistics
    int64_t n_submitted = 0, n_completed = 0, n_rejected = 0, samples_done = 0, steps = 0;
    double first_submit = -1, last_done = 0, busy_s = 0;
    std::vector<double> lat;

    void admit_locked();
    void activate_rounds_locked();
    bool build_step_locked(int b);
    void add_chunk_locked(StepBuf &B, int64_t id, int64_t c);
    scc_status launch_step(int b);
    void complete_step_locked(int b, std::unique_lock<std::mutex> &lk);
    void run();
};

// admission, in submission order: a request enters when its outputs fit the arena
void scc_server::admit_locked()
{
    while (!pending.empty() && (int)active.size() < max_active) {
        Request &r = reqs[pending.front()];
        const int64_t off = arena.alloc(r.bytes);
        if (off < 0) break;
        pending.pop_front();
        r.off = off;
        r.admitted = true;
        r.t_admit = now_s(t0);
        uint8_t *p = arena_base + off;
        const int64_t n = r.q.n;
        r.verts = (int32_t *)p;
        r.cls = (uint32_t *)(p + Arena::round((int64_t)n * r.k * 4));
        r.par = (int8_t *)((uint8_t *)r.cls + Arena::round(n * 4));
        if (r.q.kind == SCC_REQ_AGS_ROUND) {
            sessions[r.q.session].rounds.push_back(r.id);
        } else {
            r.shape = r.q.shape;
            r.seed = r.q.seed;
            r.stream = r.q.stream_id;
            r.first = r.q.first_index;
            if (!r.q.classify) r.cls = nullptr;
            active.push_back(r.id);
        }
    }
}

// an AGS round becomes active when its session has no round in progress
void scc_server::activate_rounds_locked()
{
    for (Session &s : sessions) {
        if (s.busy || s.rounds.empty() || (int)active.size() >= max_active) continue;
        Request &r = reqs[s.rounds.front()];
        s.rounds.pop_front();
        r.shape = s.st.j;
        r.seed = s.seed;
        r.stream = s.stream;
        r.first = s.next_first;
        s.next_first += (uint64_t)r.q.n;
        s.busy = true;
        // this round's class histogram, cleared before any of its steps (on either stream) runs
        (void)hipMemsetAsync(s.dhist, 0, (size_t)s.st.S * 8, side);
        (void)hipStreamSynchronize(side);
        active.push_back(r.id);
    }
}

// chunks of the next step: one per active request with unassigned rows, round
// robin, each up to max(chunk, its weighted share of the step); FIFO mode: the
// oldest request, whole
bool scc_server::build_step_locked(int b)
{
    StepBuf &B = sb[b];
    B.req.clear();
    B.nch = 0;
    B.total = 0;
    std::vector<int64_t> cand;
    for (int64_t id : active) {
        const Request &r = reqs[id];
        if (r.assigned < r.q.n) cand.push_back(id);
    }
    if (cand.empty()) return false;
    if (o.fifo) {
        const int64_t id = *std::min_element(cand.begin(), cand.end());
        cand.assign(1, id);
    }
    if (o.small_request > 0 && !o.fifo) {
        // small requests first (whole), then the others in arrival order (ids
        // increase with submission), each taking what the step still holds; a
        // step holding a small request is cut to small_step samples, so that a
        // small request waits for short steps only
        std::vector<int64_t> small, large;
        for (int64_t id : cand) (reqs[id].q.n <= o.small_request ? small : large).push_back(id);
        std::sort(small.begin(), small.end());
        std::sort(large.begin(), large.end());
        const int64_t cap = !small.empty() && o.small_step > 0 ? std::min(o.small_step, o.step_samples) : o.step_samples;
        small.insert(small.end(), large.begin(), large.end());
        for (int64_t id : small) {
            if (B.total >= cap) break;
            Request &r = reqs[id];
            const int64_t c = std::min(cap - B.total, r.q.n - r.assigned);
            add_chunk_locked(B, id, c);
        }
        return true;
    }
    // weighted shares of the step: an AGS round (which holds up its session's later
    // rounds) weighs ags_weight, a sample request 1, times 1 + age / age_tau when
    // age weighting is on; every share is at least `chunk`
    const double tnow = now_s(t0);
    auto weight = [&](const Request &r) {
        const double w = r.q.kind == SCC_REQ_AGS_ROUND ? o.ags_weight : 1.0;
        return o.age_tau > 0 ? w * (1.0 + (tnow - r.t_submit) / o.age_tau) : w;
    };
    double wsum = 0;
    for (int64_t id : cand) wsum += weight(reqs[id]);
    const size_t nc = cand.size();
    for (size_t q = 0; q < nc; q++) {
        const int64_t id = cand[(rr + q) % nc];
        Request &r = reqs[id];
        const double w = weight(r);
        const int64_t quota = o.fifo ? INT64_MAX
                                     : std::max<int64_t>(o.chunk, (int64_t)((double)o.step_samples * w / wsum));
        const int64_t c = std::min(quota, r.q.n - r.assigned);
        add_chunk_locked(B, id, c);
        if (B.total >= o.step_samples && !o.fifo) break;
    }
    rr = (rr + 1) % std::max<size_t>(1, nc);
    return true;
}

// the next c rows of request id as one chunk of step buffer B
void scc_server::add_chunk_locked(StepBuf &B, int64_t id, int64_t c)
{
    Request &r = reqs[id];
    if (r.assigned == 0) r.t_start = now_s(t0);
    const int a = B.nch;
    SampleArgs A = base[r.q.table][r.shape + 1];
    A.seed = r.seed; A.stream = r.stream; A.first = r.first; A.nsamp = r.q.n;
    A.verts = r.verts; A.par = r.par; A.err = B.derr;
    B.hargs[a] = A;
    ServeClassArgs C{};
    const scc_table *T = tables[r.q.table];
    C.g = GraphView{T->n, T->row_ptr, T->col_idx, T->colors};
    C.k = T->k;
    C.nclass = (uint32_t)nclass[r.q.table];
    C.lut = lut[r.q.table];
    C.verts = r.verts;
    C.cls = r.cls;
    C.hist = r.q.kind == SCC_REQ_AGS_ROUND ? sessions[r.q.session].dhist : nullptr;
    B.hcls[a] = C;
    B.hch[a] = ServeChunk{a, 0, r.assigned, c};
    B.total += c;
    B.hend[a] = B.total;
    B.req.push_back(id);
    B.nch++;
    r.assigned += c;
}

scc_status scc_server::launch_step(int b)
{
    StepBuf &B = sb[b];
    const int n = B.nch;
    hipStream_t st = B.stream;
    HIP_TRY(hipMemsetAsync(B.derr, 0, 4, st));
    HIP_TRY(hipMemcpyAsync(B.dargs, B.hargs, (size_t)n * sizeof(SampleArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B.dcls, B.hcls, (size_t)n * sizeof(ServeClassArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B.dch, B.hch, (size_t)n * sizeof(ServeChunk), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B.dend, B.hend, (size_t)n * 8, hipMemcpyHostToDevice, st));
    launch_serve_sample(B.dargs, B.dch, B.dend, n, B.total, B.derr, o.grid, st);
    launch_serve_classify(B.dcls, B.dch, B.dend, n, B.total, st);
    HIP_TRY(hipMemcpyAsync(B.herr, B.derr, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(B.ev, st));
    HIP_TRY(hipGetLastError());
    return SCC_OK;
}

// rows of step b are done: finish requests whose rows are all done; an AGS
// round reads its class histogram and advances its session first, and only
// then is marked finished (a finished request may be released by a caller)
void scc_server::complete_step_locked(int b, std::unique_lock<std::mutex> &lk)
{
    StepBuf &B = sb[b];
    const double t = now_s(t0);
    const int err = *B.herr;
    auto finish = [&](Request &r) {
        r.finished = true;
        r.t_done = t;
        n_completed++;
        samples_done += r.q.n;
        last_done = t;
        lat.push_back(r.t_done - r.t_submit);
    };
    std::vector<int64_t> rounds;
    for (int c = 0; c < B.nch; c++) {
        Request &r = reqs[B.req[c]];
        r.done += B.hch[c].count;
        if (err) r.status = SCC_EDEVICE;
        if (r.done < r.q.n) continue;
        active.erase(std::find(active.begin(), active.end(), r.id));
        if (r.q.kind == SCC_REQ_AGS_ROUND) rounds.push_back(r.id);
        else finish(r);
    }
    for (int64_t id : rounds) {
        // the histogram copy runs without the lock: the request is not finished
        // yet, so no caller can release it, and sessions live in a deque, whose
        // elements keep their addresses when sessions are opened meanwhile
        Session &s = sessions[reqs.at(id).q.session];
        unsigned long long *dst = s.hh.data();
        const unsigned long long *src = s.dhist;
        const size_t bytes = (size_t)s.st.S * 8;
        lk.unlock();
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, side);
        if (e == hipSuccess) e = hipStreamSynchronize(side);
        lk.lock();
        Request &r = reqs.at(id);
        if (e != hipSuccess) r.status = SCC_EDEVICE;
        else if (r.status == SCC_OK) s.st.add_round(r.q.n, s.hh.data());
        s.busy = false;
        finish(r);
    }
    steps++;
    cv_done.notify_all();
}

void scc_server::run()
{
    std::unique_lock<std::mutex> lk(mu);
    bool busy[STEP_BUFS] = {};
    for (;;) {
        admit_locked();
        activate_rounds_locked();
        int nbusy = 0, free_b = -1;
        for (int b = 0; b < STEP_BUFS; b++) {
            if (busy[b]) nbusy++;
            else if (free_b < 0) free_b = b;
        }
        if (stop && nbusy == 0) break;
        // a free buffer and work: launch a step on that buffer's stream
        // the first-in first-out mode runs one request at a time: one step in flight
        const int max_inflight = o.fifo ? 1 : STEP_BUFS;
        if (!stop && free_b >= 0 && nbusy < max_inflight && build_step_locked(free_b)) {
            lk.unlock();
            const scc_status s = launch_step(free_b);
            lk.lock();
            if (s) {
                fatal = s;
                for (int64_t id : sb[free_b].req) reqs[id].status = s;
            }
            busy[free_b] = true;
            continue;
        }
        if (nbusy) {
            // finish whichever step is done first (the two streams overlap)
            lk.unlock();
            int done = -1;
            hipError_t e = hipSuccess;
            const auto w0 = std::chrono::steady_clock::now();
            while (done < 0) {
                for (int b = 0; b < STEP_BUFS && done < 0; b++) {
                    if (!busy[b]) continue;
                    const hipError_t q = hipEventQuery(sb[b].ev);
                    if (q == hipErrorNotReady) continue;
                    done = b;
                    e = q;
                }
                if (done < 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
            const double waited = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
            lk.lock();
            busy_s += waited;
            busy[done] = false;
            if (e != hipSuccess) {
                fatal = SCC_EDEVICE;
                for (int64_t id : sb[done].req) reqs[id].status = SCC_EDEVICE;
            }
            complete_step_locked(done, lk);
            continue;
        }
        cv_work.wait_for(lk, std::chrono::milliseconds(20));
    }
    // requests that will not run any more
    for (auto &kv : reqs)
        if (!kv.second.finished) { kv.second.finished = true; kv.second.status = SCC_EBUSY; }
    cv_done.notify_all();
}

extern "C" scc_status scc_server_create(const scc_server_opts *opts, scc_server **out)
{
    if (!opts || !out) return set_error(SCC_EINVAL, "NULL argument");
    *out = nullptr;
    if (opts->n_tables < 1 || !opts->tables) return set_error(SCC_EINVAL, "no tables");
    for (int i = 0; i < opts->n_tables; i++)
        if (!opts->tables[i]) return set_error(SCC_EINVAL, "table %d is NULL", i);
    auto *S = new scc_server();
    S->o = *opts;
    if (S->o.hbm_budget <= 0) S->o.hbm_budget = (int64_t)1 << 30;
    if (S->o.max_pending <= 0) S->o.max_pending = 4096;
    if (S->o.max_active <= 0) S->o.max_active = 256;
    if (S->o.step_samples <= 0) S->o.step_samples = (int64_t)1 << 18;
    if (S->o.chunk <= 0) S->o.chunk = 8192;
    if (S->o.grid <= 0) S->o.grid = 8192;
    if (!(S->o.ags_weight > 0)) S->o.ags_weight = 1.0;
    S->max_active = S->o.max_active;
    S->mem.alloc = S->o.alloc;
    auto fail = [&](scc_status s) {
        scc_server_destroy(S);
        return s;
    };
    if (S->o.stream) {
        S->st = (hipStream_t)S->o.stream;
    } else {
        if (hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess)
            return fail(set_error(SCC_EDEVICE, "server stream"));
        S->own_stream = true;
    }
    S->mem.stream = S->st;
    if (hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->st2, hipStreamNonBlocking) != hipSuccess)
        return fail(set_error(SCC_EDEVICE, "server streams"));
    S->sb[0].stream = S->st;
    S->sb[1].stream = S->st2;
    // everything the loop needs is built and allocated here, on the caller's thread
    for (int i = 0; i < opts->n_tables; i++) {
        scc_table *T = const_cast<scc_table *>(opts->tables[i]);
        S->tables.push_back(T);
        scc_status s = prepare_all_sampling(T);
        if (s) return fail(s);
        std::vector<SampleArgs> b(T->hlut.num_unr + 1);
        for (int shape = -1; shape < T->hlut.num_unr; shape++) {
            SampleArgs A{};
            if (sample_weight(T, shape) > 0) {
                s = prepare_sampling(T, shape, &A);
                if (s) return fail(s);
            }
            b[shape + 1] = A;
        }
        S->base.push_back(b);
        const uint16_t *l;
        int nc;
        s = class_lut(T->k, S->st, &l, &nc);
        if (s) return fail(s);
        S->lut.push_back(l);
        S->nclass.push_back(nc);
    }
    S->arena_base = (uint8_t *)S->mem.get((size_t)S->o.hbm_budget);
    if (!S->arena_base) return fail(set_error(SCC_ENOMEM, "server arena of %lld bytes", (long long)S->o.hbm_budget));
    S->arena.reset(S->o.hbm_budget);
    const int na = S->max_active;
    for (StepBuf &B : S->sb) {
        if (hipHostMalloc((void **)&B.hargs, (size_t)na * sizeof(SampleArgs)) != hipSuccess ||
            hipHostMalloc((void **)&B.hcls, (size_t)na * sizeof(ServeClassArgs)) != hipSuccess ||
            hipHostMalloc((void **)&B.hch, (size_t)na * sizeof(ServeChunk)) != hipSuccess ||
            hipHostMalloc((void **)&B.hend, (size_t)na * 8) != hipSuccess ||
            hipHostMalloc((void **)&B.herr, 64) != hipSuccess)
            return fail(set_error(SCC_ENOMEM, "server host buffers"));
        B.dargs = (SampleArgs *)S->mem.get((size_t)na * sizeof(SampleArgs));
        B.dcls = (ServeClassArgs *)S->mem.get((size_t)na * sizeof(ServeClassArgs));
        B.dch = (ServeChunk *)S->mem.get((size_t)na * sizeof(ServeChunk));
        B.dend = (int64_t *)S->mem.get((size_t)na * 8);
        B.derr = (int *)S->mem.get(64);
        if (!B.dargs || !B.dcls || !B.dch || !B.dend || !B.derr) return fail(set_error(SCC_ENOMEM, "server step buffers"));
        if (hipEventCreateWithFlags(&B.ev, hipEventDisableTiming) != hipSuccess)
            return fail(set_error(SCC_EDEVICE, "server events"));
    }
    if (hipStreamSynchronize(S->st) != hipSuccess) return fail(set_error(SCC_EDEVICE, "server set-up"));
    S->t0 = std::chrono::steady_clock::now();
    S->th = std::thread([S] { S->run(); });
    *out = S;
    return SCC_OK;
}

extern "C" scc_status scc_server_ags_open(scc_server *S, int table, int64_t cbar, uint64_t seed, uint64_t stream_id,
                                          int *session)
{
    if (!S || !session) return set_error(SCC_EINVAL, "NULL argument");
    if (table < 0 || table >= (int)S->tables.size()) return set_error(SCC_EINVAL, "table %d out of range", table);
    if (cbar < 1) return set_error(SCC_EINVAL, "cbar < 1");
    if (S->tables[table]->rooting == SCC_ROOT_BALANCED)
        return set_error(SCC_EINVAL, "AGS sessions need zero-rooting or all rootings");
    Session s;
    s.table = table;
    s.seed = seed;
    s.stream = stream_id;
    scc_status r = s.st.init(S->tables[table], cbar, S->side);
    if (r) return r;
    s.hh.assign(s.st.S, 0);
    s.dhist = (unsigned long long *)S->mem.get((size_t)s.st.S * 8 + 64);
    if (!s.dhist) return set_error(SCC_ENOMEM, "AGS histogram");
    std::lock_guard<std::mutex> lk(S->mu);
    S->sessions.push_back(std::move(s));
    *session = (int)S->sessions.size() - 1;
    return SCC_OK;
}

extern "C" scc_status scc_server_ags_result(scc_server *S, int session, int64_t *hits, double *w, int64_t *n_j,
                                            int32_t *round_shapes, int64_t cap, int64_t *n_rounds)
{
    if (!S || !hits || !w || !n_j || !n_rounds) return set_error(SCC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (session < 0 || session >= (int)S->sessions.size()) return set_error(SCC_EINVAL, "no session %d", session);
    const Session &s = S->sessions[session];
    s.st.result(hits, w, n_j);
    *n_rounds = (int64_t)s.st.shapes.size();
    if (round_shapes)
        for (int64_t r = 0; r < std::min<int64_t>(cap, *n_rounds); r++) round_shapes[r] = s.st.shapes[r];
    return SCC_OK;
}

extern "C" scc_status scc_server_submit(scc_server *S, const scc_request *q, int64_t *id)
{
    if (!S || !q || !id) return set_error(SCC_EINVAL, "NULL argument");
    if (q->table < 0 || q->table >= (int)S->tables.size()) return set_error(SCC_EINVAL, "table %d out of range", q->table);
    if (q->n < 1) return set_error(SCC_EINVAL, "n < 1");
    const scc_table *T = S->tables[q->table];
    if (q->kind == SCC_REQ_SAMPLE) {
        if (q->shape < -1 || q->shape >= T->hlut.num_unr) return set_error(SCC_EINVAL, "shape %d out of range", q->shape);
        if (sample_weight(T, q->shape) == 0)
            return set_error(SCC_EEMPTY, "no colourful %d-treelet of this shape", T->k);
    } else if (q->kind == SCC_REQ_AGS_ROUND) {
        std::lock_guard<std::mutex> lk(S->mu);
        if (q->session < 0 || q->session >= (int)S->sessions.size())
            return set_error(SCC_EINVAL, "no AGS session %d", q->session);
        if (S->sessions[q->session].table != q->table)
            return set_error(SCC_EINVAL, "session %d samples table %d", q->session, S->sessions[q->session].table);
    } else {
        return set_error(SCC_EINVAL, "unknown request kind %d", q->kind);
    }
    Request r;
    r.q = *q;
    r.k = T->k;
    r.bytes = Arena::round(q->n * T->k * 4) + Arena::round(q->n * 4) + Arena::round(q->n * T->k);
    if (r.bytes > S->o.hbm_budget)
        return set_error(SCC_ENOMEM, "a request of %lld samples needs %lld bytes, over the budget", (long long)q->n,
                         (long long)r.bytes);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) return set_error((scc_status)S->fatal, "the server stopped after a device error");
    if ((int)S->pending.size() >= S->o.max_pending) {
        S->n_rejected++;
        return set_error(SCC_EBUSY, "server full: %d requests wait for admission", (int)S->pending.size());
    }
    r.id = S->next_id++;
    r.t_submit = now_s(S->t0);
    if (S->first_submit < 0) S->first_submit = r.t_submit;
    S->reqs[r.id] = r;
    S->pending.push_back(r.id);
    S->n_submitted++;
    *id = r.id;
    S->cv_work.notify_one();
    return SCC_OK;
}

extern "C" scc_status scc_server_wait(scc_server *S, int64_t id, double timeout_s, scc_result *out)
{
    if (!S || !out) return set_error(SCC_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return set_error(SCC_EINVAL, "no request %lld", (long long)id);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (!S->reqs[id].finished) {
        if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !S->reqs[id].finished)
            return set_error(SCC_EBUSY, "request %lld not finished", (long long)id);
    }
    const Request &r = S->reqs[id];
    memset(out, 0, sizeof *out);
    out->id = r.id;
    out->status = r.status;
    out->k = r.k;
    out->shape = r.shape;
    out->n = r.q.n;
    out->first_index = r.first;
    out->verts = r.verts;
    out->parent = r.par;
    out->cls = r.cls;
    out->t_submit = r.t_submit;
    out->t_admit = r.t_admit;
    out->t_start = r.t_start;
    out->t_done = r.t_done;
    return SCC_OK;
}

extern "C" scc_status scc_server_release(scc_server *S, int64_t id)
{
    if (!S) return set_error(SCC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return set_error(SCC_EINVAL, "no request %lld", (long long)id);
    if (!it->second.finished) return set_error(SCC_EBUSY, "request %lld still running", (long long)id);
    if (it->second.off >= 0) S->arena.release(it->second.off, it->second.bytes);
    S->reqs.erase(it);
    S->cv_work.notify_one();
    return SCC_OK;
}

extern "C" scc_status scc_server_get_stats(scc_server *S, scc_server_stats *out)
{
    if (!S || !out) return set_error(SCC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    memset(out, 0, sizeof *out);
    out->submitted = S->n_submitted;
    out->completed = S->n_completed;
    out->rejected = S->n_rejected;
    out->samples = S->samples_done;
    out->steps = S->steps;
    out->arena_peak = S->arena.peak();
    out->arena_used = S->arena.used();
    out->busy_s = S->busy_s;
    out->span_s = S->first_submit >= 0 ? S->last_done - S->first_submit : 0.0;
    if (!S->lat.empty()) {
        std::vector<double> l = S->lat;
        std::sort(l.begin(), l.end());
        auto q = [&](double p) {
            const size_t i = (size_t)std::min<double>((double)l.size() - 1, std::ceil(p * (double)l.size()) - 1);
            return l[i] * 1e3;
        };
        out->p50_ms = q(0.50);
        out->p99_ms = q(0.99);
        double s = 0;
        for (double x : l) s += x;
        out->mean_ms = s / (double)l.size() * 1e3;
        out->max_ms = l.back() * 1e3;
    }
    return SCC_OK;
}

extern "C" void scc_server_destroy(scc_server *S)
{
    if (!S) return;
    if (S->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        S->th.join();
    }
    if (S->st) (void)hipStreamSynchronize(S->st);
    if (S->st2) (void)hipStreamSynchronize(S->st2);
    if (S->side) (void)hipStreamSynchronize(S->side);
    for (StepBuf &B : S->sb) {
        if (B.hargs) (void)hipHostFree(B.hargs);
        if (B.hcls) (void)hipHostFree(B.hcls);
        if (B.hch) (void)hipHostFree(B.hch);
        if (B.hend) (void)hipHostFree(B.hend);
        if (B.herr) (void)hipHostFree(B.herr);
        S->mem.put(B.dargs); S->mem.put(B.dcls); S->mem.put(B.dch); S->mem.put(B.dend); S->mem.put(B.derr);
        if (B.ev) (void)hipEventDestroy(B.ev);
    }
    for (Session &s : S->sessions) S->mem.put(s.dhist);
    S->mem.put(S->arena_base);
    if (S->st) (void)hipStreamSynchronize(S->st);
    if (S->side) (void)hipStreamDestroy(S->side);
    if (S->st2) (void)hipStreamDestroy(S->st2);
    if (S->own_stream && S->st) (void)hipStreamDestroy(S->st);
    delete S;
}
