// serving.hip -- fold-in serving engine (bpmf_server_* in include/bpmf.h).
//
// Continuous batching: a dispatcher thread owns n_streams slots, each with a
// device buffer and a pinned host staging buffer holding one batch.  When a
// slot is free it takes queued requests in arrival order while the batch
// fits the slot (memory admission), the batch-size cap and the global
// in-flight cap, packs them in CSR form, and enqueues upload -> bpmf_foldin
// -> download -> event on the slot's stream.  Slots run concurrently, so
// uploads, kernels and downloads of different batches overlap; a request that
// arrives while others are on the GPU waits only for the next free slot.
// Each request's predictions are computed independently of its batch mates.
//
// Resident mode (bpmf_server_create_resident): no launch or copy per
// request.  A persistent kernel (kernels_resident.hip) owns n_slots request
// slots in coherent pinned host memory; the dispatcher writes a queued
// request into a free slot and bumps its sequence number, the kernel writes
// the predictions back into the slot, and the dispatcher collects them.  The
// kernel ends after about a second without requests (or on the stop flag);
// the dispatcher launches it again whenever a request waits and it is not
// running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bpmf.h"
#include "resident.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    int64_t id;
    std::vector<int32_t> cols;
    std::vector<float> vals;
    std::vector<int32_t> qcols;
    Clock::time_point t_submit;
};

struct Done {
    int64_t id;
    std::vector<float> preds;
    double latency;
};

constexpr size_t kAlign = 256;

size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Device bytes of a batch with B requests, nnz ratings and nq queries:
// [req_ptr][q_ptr][cols][qcols][vals][out][per-sample partials].
size_t batch_bytes(int64_t B, int64_t nnz, int64_t nq, int S)
{
    return al(8 * (B + 1)) + al(8 * (B + 1)) + al(4 * nnz) + al(4 * nq) + al(4 * nnz) + al(4 * nq) +
           al(4 * (size_t)S * std::max<int64_t>(nq, 1));
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char *d_buf = nullptr;
    char *h_buf = nullptr;   // pinned: packed inputs
    float *h_out = nullptr;  // pinned: predictions
    std::vector<Req> batch;
    std::vector<int64_t> q_off;
    bool busy = false;
};

}  // namespace

struct bpmf_server {
    bpmf_foldin_model m;
    size_t capacity = 0;  // bytes per slot
    int max_batch = 0, max_inflight = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    std::deque<Req> queue;
    std::deque<Done> done;
    int64_t submitted = 0, completed = 0;
    int inflight = 0;
    bpmf_server_stats stats{};
    std::atomic<bool> stop{false};
    int device = 0;
    std::thread worker;
    std::string error;
    // resident mode
    bool resident = false;
    int n_slots = 0, max_nnz = 0, max_q = 0;
    int64_t idle_polls = 0;
    size_t r_slot_bytes = 0;
    char *r_slots = nullptr;          // coherent pinned host memory
    int32_t *r_stop = nullptr;        // coherent pinned host memory
    char *r_dev = nullptr;            // device staging
    hipStream_t r_stream = nullptr;
    hipStream_t r_fb_stream = nullptr;  // FP64 recompute of requests whose FP32 pivot failed
    std::vector<Req> r_req;
    std::vector<int32_t> r_seq;
    std::vector<char> r_busy;
};

static bpmf_status srv_fail(bpmf_status s, const std::string &m)
{
    bpmf::set_last_error(m);
    return s;
}

static bool launch_batch(bpmf_server *srv, Slot &sl)
{
    const int S = srv->m.S;
    const int64_t B = (int64_t)sl.batch.size();
    int64_t nnz = 0, nq = 0;
    for (auto &r : sl.batch) {
        nnz += (int64_t)r.cols.size();
        nq += (int64_t)r.qcols.size();
    }
    size_t o = 0;
    const size_t o_rp = o; o += al(8 * (B + 1));
    const size_t o_qp = o; o += al(8 * (B + 1));
    const size_t o_c = o; o += al(4 * nnz);
    const size_t o_qc = o; o += al(4 * nq);
    const size_t o_v = o; o += al(4 * nnz);
    const size_t in_bytes = o;
    const size_t o_out = o; o += al(4 * nq);
    const size_t o_ws = o; o += al(4 * (size_t)S * std::max<int64_t>(nq, 1));
    int64_t *rp = (int64_t *)(sl.h_buf + o_rp);
    int64_t *qp = (int64_t *)(sl.h_buf + o_qp);
    int32_t *c = (int32_t *)(sl.h_buf + o_c);
    int32_t *qc = (int32_t *)(sl.h_buf + o_qc);
    float *v = (float *)(sl.h_buf + o_v);
    rp[0] = 0;
    qp[0] = 0;
    sl.q_off.assign(B + 1, 0);
    for (int64_t i = 0; i < B; ++i) {
        const Req &r = sl.batch[i];
        std::memcpy(c + rp[i], r.cols.data(), 4 * r.cols.size());
        std::memcpy(v + rp[i], r.vals.data(), 4 * r.vals.size());
        std::memcpy(qc + qp[i], r.qcols.data(), 4 * r.qcols.size());
        rp[i + 1] = rp[i] + (int64_t)r.cols.size();
        qp[i + 1] = qp[i] + (int64_t)r.qcols.size();
        sl.q_off[i + 1] = qp[i + 1];
    }
    char *d = sl.d_buf;
    if (hipMemcpyAsync(d, sl.h_buf, in_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess) return false;
    bpmf_status st = bpmf_foldin(&srv->m, B, (const int64_t *)(d + o_rp), (const int32_t *)(d + o_c),
                                 (const float *)(d + o_v), (const int64_t *)(d + o_qp),
                                 (const int32_t *)(d + o_qc), nq, (float *)(d + o_out), d + o_ws,
                                 o - o_ws, sl.stream);
    if (st != BPMF_OK) return false;
    if (nq > 0 && hipMemcpyAsync(sl.h_out, d + o_out, 4 * nq, hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
        return false;
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return false;
    sl.busy = true;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.batches += 1;
    srv->stats.max_batch = std::max<int64_t>(srv->stats.max_batch, B);
    srv->stats.max_batch_bytes = std::max<int64_t>(srv->stats.max_batch_bytes, (int64_t)o);
    return true;
}

static void worker_loop(bpmf_server *srv)
{
    const int S = srv->m.S;
    hipSetDevice(srv->device);
    while (true) {
        bool progress = false;
        bool any_busy = false;
        // completions
        for (auto &sl : srv->slots) {
            if (!sl.busy) continue;
            if (hipEventQuery(sl.done) != hipSuccess) {
                any_busy = true;
                continue;
            }
            const auto t = Clock::now();
            std::lock_guard<std::mutex> lk(srv->mu);
            for (size_t i = 0; i < sl.batch.size(); ++i) {
                Req &r = sl.batch[i];
                Done dn;
                dn.id = r.id;
                dn.preds.assign(sl.h_out + sl.q_off[i], sl.h_out + sl.q_off[i + 1]);
                dn.latency = std::chrono::duration<double>(t - r.t_submit).count();
                srv->done.push_back(std::move(dn));
            }
            srv->completed += (int64_t)sl.batch.size();
            srv->stats.requests_done += (int64_t)sl.batch.size();
            srv->inflight -= (int)sl.batch.size();
            sl.batch.clear();
            sl.busy = false;
            progress = true;
            srv->cv_done.notify_all();
        }
        // launches
        for (auto &sl : srv->slots) {
            if (sl.busy) continue;
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                int64_t B = 0, nnz = 0, nq = 0;
                while (!srv->queue.empty() && (int)B < srv->max_batch && srv->inflight + B < srv->max_inflight) {
                    const Req &r = srv->queue.front();
                    const size_t need = batch_bytes(B + 1, nnz + (int64_t)r.cols.size(),
                                                    nq + (int64_t)r.qcols.size(), S);
                    if (need > srv->capacity) break;
                    nnz += (int64_t)r.cols.size();
                    nq += (int64_t)r.qcols.size();
                    sl.batch.push_back(std::move(srv->queue.front()));
                    srv->queue.pop_front();
                    ++B;
                }
                srv->inflight += (int)B;
                srv->stats.max_inflight = std::max<int64_t>(srv->stats.max_inflight, srv->inflight);
            }
            if (sl.batch.empty()) continue;
            if (!launch_batch(srv, sl)) {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->error = std::string("batch launch failed: ") + bpmf_last_error();
                srv->stop = true;
                srv->cv_done.notify_all();
                return;
            }
            progress = true;
            any_busy = true;
        }
        if (srv->stop) {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->queue.empty() && !any_busy) return;
        }
        if (!progress) {
            if (any_busy) {
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> lk(srv->mu);
                srv->cv_submit.wait_for(lk, std::chrono::milliseconds(1),
                                        [&] { return !srv->queue.empty() || srv->stop; });
            }
        }
    }
}

// Device staging of the resident server: cols and vals (max_nnz per slot),
// query columns (max_q per slot), Lambda_s mu_s (S x K), then one batch of
// bpmf_foldin for a single request of at most max_nnz ratings and max_q
// queries (the FP64 recompute of a request whose FP32 pivot failed).
static size_t resident_dev_bytes(int32_t n_slots, int32_t max_nnz, int32_t max_q, int S, int K)
{
    return 2 * al(4 * (size_t)n_slots * max_nnz) + al(4 * (size_t)n_slots * max_q) + al(4 * (size_t)S * K) +
           batch_bytes(1, max_nnz, max_q, S);
}

static float *resident_lam_mu(bpmf_server *srv)
{
    return (float *)(srv->r_dev + 2 * al(4 * (size_t)srv->n_slots * srv->max_nnz) +
                     al(4 * (size_t)srv->n_slots * srv->max_q));
}

static char *resident_fallback_buf(bpmf_server *srv)
{
    return (char *)resident_lam_mu(srv) + al(4 * (size_t)srv->m.S * srv->m.K);
}

// The resident kernel has no FP64 path: a (request, sample) pair whose FP32
// pivot fails comes back as NaN predictions.  Such a request is computed
// again by bpmf_foldin, which takes the pairs that pass in FP32 with the same
// arithmetic as the resident kernel and recomputes the failed ones in FP64,
// so its predictions are those of batching mode.  Rare: the dispatcher waits
// for it on a stream of its own.
static bool resident_recompute(bpmf_server *srv, const Req &r, std::vector<float> &preds)
{
    const int64_t nnz = (int64_t)r.cols.size(), nq = (int64_t)r.qcols.size();
    char *d = resident_fallback_buf(srv);
    const size_t o_rp = 0, o_qp = o_rp + al(16), o_c = o_qp + al(16), o_qc = o_c + al(4 * nnz),
                 o_v = o_qc + al(4 * nq), o_out = o_v + al(4 * nnz), o_ws = o_out + al(4 * nq);
    const int64_t rp[2] = {0, nnz}, qp[2] = {0, nq};
    hipStream_t st = srv->r_fb_stream;
    if (hipMemcpyAsync(d + o_rp, rp, 16, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d + o_qp, qp, 16, hipMemcpyHostToDevice, st) != hipSuccess ||
        (nnz > 0 && hipMemcpyAsync(d + o_c, r.cols.data(), 4 * nnz, hipMemcpyHostToDevice, st) != hipSuccess) ||
        (nnz > 0 && hipMemcpyAsync(d + o_v, r.vals.data(), 4 * nnz, hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(d + o_qc, r.qcols.data(), 4 * nq, hipMemcpyHostToDevice, st) != hipSuccess)
        return false;
    if (bpmf_foldin(&srv->m, 1, (const int64_t *)(d + o_rp), (const int32_t *)(d + o_c), (const float *)(d + o_v),
                    (const int64_t *)(d + o_qp), (const int32_t *)(d + o_qc), nq, (float *)(d + o_out), d + o_ws,
                    al(4 * (size_t)srv->m.S * std::max<int64_t>(nq, 1)), st) != BPMF_OK)
        return false;
    std::vector<float> out(nq);
    if (hipMemcpyAsync(out.data(), d + o_out, 4 * nq, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return false;
    preds.swap(out);
    return true;
}

static bpmf::ResidentArgs resident_args(bpmf_server *srv)
{
    bpmf::ResidentArgs ra;
    ra.slots = srv->r_slots;
    ra.slot_bytes = (int64_t)srv->r_slot_bytes;
    ra.max_nnz = srv->max_nnz;
    ra.max_q = srv->max_q;
    ra.stop = srv->r_stop;
    ra.dev_cols = (int32_t *)srv->r_dev;
    ra.dev_vals = (float *)(srv->r_dev + al(4 * (size_t)srv->n_slots * srv->max_nnz));
    ra.dev_q = (int32_t *)(srv->r_dev + 2 * al(4 * (size_t)srv->n_slots * srv->max_nnz));
    ra.lam_mu = resident_lam_mu(srv);
    ra.idle_polls = srv->idle_polls;
    return ra;
}

static hipError_t resident_launch(bpmf_server *srv)
{
    const bpmf_foldin_model &m = srv->m;
    return bpmf::launch_resident(srv->n_slots, m.S, m.K, m.N, m.alpha, m.mean_rating, m.d_V, m.d_Lambda, m.d_mu,
                                 resident_args(srv), srv->r_stream);
}

static bpmf::ResidentSlotHeader *slot_header(bpmf_server *srv, int i)
{
    return (bpmf::ResidentSlotHeader *)(srv->r_slots + (size_t)i * srv->r_slot_bytes);
}

static void resident_loop(bpmf_server *srv)
{
    hipSetDevice(srv->device);
    int relaunches = 0;  // launches since the last completed request
    while (true) {
        bool progress = false, any_busy = false;
        // completions
        for (int i = 0; i < srv->n_slots; ++i) {
            if (!srv->r_busy[i]) continue;
            bpmf::ResidentSlotHeader *h = slot_header(srv, i);
            if (__atomic_load_n(&h->done_seq, __ATOMIC_ACQUIRE) != srv->r_seq[i]) {
                any_busy = true;
                continue;
            }
            const auto t = Clock::now();
            const float *out = (const float *)((char *)h + bpmf::RESIDENT_HEADER_BYTES +
                                               8 * (size_t)srv->max_nnz + 4 * (size_t)srv->max_q);
            Req &r = srv->r_req[i];
            Done dn;
            dn.id = r.id;
            dn.preds.assign(out, out + r.qcols.size());
            bool nan_seen = false;
            for (float v : dn.preds) nan_seen |= std::isnan(v);
            if (nan_seen) resident_recompute(srv, r, dn.preds);
            dn.latency = std::chrono::duration<double>(t - r.t_submit).count();
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->done.push_back(std::move(dn));
            srv->completed += 1;
            srv->stats.requests_done += 1;
            srv->inflight -= 1;
            srv->r_busy[i] = 0;
            progress = true;
            relaunches = 0;
            srv->cv_done.notify_all();
        }
        // free slots take queued requests in arrival order
        for (int i = 0; i < srv->n_slots; ++i) {
            if (srv->r_busy[i]) continue;
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                if (srv->queue.empty()) break;
                srv->r_req[i] = std::move(srv->queue.front());
                srv->queue.pop_front();
                srv->inflight += 1;
                srv->stats.batches += 1;
                srv->stats.max_batch = 1;
                int64_t busy = 1;
                for (int k = 0; k < srv->n_slots; ++k) busy += srv->r_busy[k] ? 1 : 0;
                srv->stats.max_inflight = std::max<int64_t>(srv->stats.max_inflight, busy);
            }
            const Req &r = srv->r_req[i];
            bpmf::ResidentSlotHeader *h = slot_header(srv, i);
            int32_t *cols = (int32_t *)((char *)h + bpmf::RESIDENT_HEADER_BYTES);
            float *vals = (float *)(cols + srv->max_nnz);
            int32_t *qc = (int32_t *)(vals + srv->max_nnz);
            std::memcpy(cols, r.cols.data(), 4 * r.cols.size());
            std::memcpy(vals, r.vals.data(), 4 * r.vals.size());
            std::memcpy(qc, r.qcols.data(), 4 * r.qcols.size());
            h->nnz = (int32_t)r.cols.size();
            h->nq = (int32_t)r.qcols.size();
            srv->r_seq[i] += 1;
            __atomic_store_n(&h->req_seq, srv->r_seq[i], __ATOMIC_RELEASE);
            __atomic_fetch_add(srv->r_stop + 1, 1, __ATOMIC_RELEASE);  // activity: no workgroup ends while requests come
            srv->r_busy[i] = 1;
            any_busy = true;
            progress = true;
        }
        // a request waits and the kernel has ended (idle timeout): launch it again
        if (any_busy && hipStreamQuery(srv->r_stream) == hipSuccess) {
            if (++relaunches > 3 || resident_launch(srv) != hipSuccess) {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->error = "resident fold-in kernel makes no progress";
                srv->stop = true;
                srv->cv_done.notify_all();
                return;
            }
        }
        if (srv->stop) {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->queue.empty() && !any_busy) return;
        }
        if (!progress) {
            if (any_busy) {
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> lk(srv->mu);
                srv->cv_submit.wait_for(lk, std::chrono::milliseconds(1),
                                        [&] { return !srv->queue.empty() || srv->stop; });
            }
        }
    }
}

extern "C" {

bpmf_status bpmf_server_create_resident(bpmf_server **out, const bpmf_foldin_model *m, int32_t n_slots,
                                        int32_t max_nnz, int32_t max_q, int64_t idle_polls)
{
    if (!out || !m) return srv_fail(BPMF_E_INVALID, "NULL argument");
    *out = nullptr;
    if (m->S < 1 || m->S > 16 || m->K < 1 || m->K > 64 || m->N < 1 || !m->d_V || !m->d_Lambda || !m->d_mu)
        return srv_fail(BPMF_E_INVALID, "bad fold-in model (resident mode: S in 1..16, K in 1..64)");
    if (n_slots < 1 || n_slots > 256 || max_nnz < 1 || max_nnz > (1 << 20) || max_q < 1 || max_q > 1024)
        return srv_fail(BPMF_E_INVALID, "n_slots in 1..256, max_nnz in 1..2^20, max_q in 1..1024");
    bpmf_server *srv = new (std::nothrow) bpmf_server();
    if (!srv) return srv_fail(BPMF_E_NOMEM, "server allocation");
    srv->m = *m;
    srv->resident = true;
    srv->n_slots = n_slots;
    srv->max_nnz = max_nnz;
    srv->max_q = max_q;
    srv->idle_polls = idle_polls > 0 ? idle_polls : 500000;
    srv->r_slot_bytes = al(bpmf::RESIDENT_HEADER_BYTES + 8 * (size_t)max_nnz + 8 * (size_t)max_q);
    srv->r_req.resize(n_slots);
    srv->r_seq.assign(n_slots, 0);
    srv->r_busy.assign(n_slots, 0);
    srv->max_batch = 1;
    srv->max_inflight = n_slots;
    srv->stats.stream_capacity = (int64_t)srv->r_slot_bytes;
    const size_t dev_bytes = resident_dev_bytes(n_slots, max_nnz, max_q, m->S, m->K);
    if (hipGetDevice(&srv->device) != hipSuccess ||
        hipStreamCreateWithFlags(&srv->r_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&srv->r_fb_stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&srv->r_slots, srv->r_slot_bytes * n_slots, hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&srv->r_stop, kAlign, hipHostMallocCoherent) != hipSuccess ||
        hipMalloc((void **)&srv->r_dev, dev_bytes) != hipSuccess ||
        bpmf::prepare_resident(m->S, m->K, m->d_Lambda, m->d_mu, resident_lam_mu(srv), srv->r_stream) != hipSuccess ||
        hipStreamSynchronize(srv->r_stream) != hipSuccess) {
        bpmf_server_destroy(srv);
        return srv_fail(BPMF_E_HIP, "resident server allocation failed");
    }
    int max_slots = 0;
    if (bpmf::resident_max_slots(m->K, m->S, &max_slots) != hipSuccess) {
        bpmf_server_destroy(srv);
        return srv_fail(BPMF_E_HIP, "resident kernel occupancy query failed");
    }
    if (n_slots > max_slots) {
        bpmf_server_destroy(srv);
        return srv_fail(BPMF_E_INVALID, "n_slots exceeds the slot workgroups the device holds at once (" +
                                            std::to_string(max_slots) + " for this S and K)");
    }
    std::memset(srv->r_slots, 0, srv->r_slot_bytes * n_slots);
    std::memset(srv->r_stop, 0, kAlign);
    if (resident_launch(srv) != hipSuccess) {
        bpmf_server_destroy(srv);
        return srv_fail(BPMF_E_HIP, "resident kernel launch failed");
    }
    srv->worker = std::thread(resident_loop, srv);
    *out = srv;
    return BPMF_OK;
}

bpmf_status bpmf_server_create(bpmf_server **out, const bpmf_foldin_model *m, size_t mem_budget_bytes,
                               int32_t n_streams, int32_t max_batch, int32_t max_inflight)
{
    if (!out || !m) return srv_fail(BPMF_E_INVALID, "NULL argument");
    *out = nullptr;
    if (m->S < 1 || m->K < 1 || m->K > 64 || m->N < 1 || !m->d_V || !m->d_Lambda || !m->d_mu)
        return srv_fail(BPMF_E_INVALID, "bad fold-in model");
    if (n_streams < 1 || n_streams > 16 || max_batch < 1 || max_inflight < 1)
        return srv_fail(BPMF_E_INVALID, "n_streams in 1..16, max_batch and max_inflight >= 1");
    const size_t cap = mem_budget_bytes / (size_t)n_streams;
    if (cap < batch_bytes(1, 1, 1, m->S)) return srv_fail(BPMF_E_INVALID, "memory budget too small");
    bpmf_server *srv = new (std::nothrow) bpmf_server();
    if (!srv) return srv_fail(BPMF_E_NOMEM, "server allocation");
    srv->m = *m;
    srv->capacity = cap;
    srv->max_batch = max_batch;
    srv->max_inflight = max_inflight;
    srv->stats.stream_capacity = (int64_t)cap;
    if (hipGetDevice(&srv->device) != hipSuccess) {
        delete srv;
        return srv_fail(BPMF_E_HIP, "hipGetDevice failed");
    }
    srv->slots.resize(n_streams);
    for (auto &sl : srv->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void **)&sl.d_buf, cap) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_buf, cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_out, cap, hipHostMallocDefault) != hipSuccess) {
            bpmf_server_destroy(srv);
            return srv_fail(BPMF_E_HIP, "stream, event or buffer allocation failed");
        }
    }
    srv->worker = std::thread(worker_loop, srv);
    *out = srv;
    return BPMF_OK;
}

bpmf_status bpmf_server_submit(bpmf_server *srv, int64_t id, int32_t nnz, const int32_t *h_cols,
                               const float *h_vals, int32_t nq, const int32_t *h_q_cols)
{
    if (!srv) return srv_fail(BPMF_E_STATE, "NULL server");
    if (nnz < 0 || nq < 0 || (nnz > 0 && (!h_cols || !h_vals)) || (nq > 0 && !h_q_cols))
        return srv_fail(BPMF_E_INVALID, "bad request arrays");
    for (int32_t i = 0; i < nnz; ++i)
        if (h_cols[i] < 0 || h_cols[i] >= srv->m.N) return srv_fail(BPMF_E_INVALID, "rating column out of range");
    for (int32_t i = 0; i < nq; ++i)
        if (h_q_cols[i] < 0 || h_q_cols[i] >= srv->m.N) return srv_fail(BPMF_E_INVALID, "query column out of range");
    if (srv->resident) {
        if (nnz > srv->max_nnz || nq > srv->max_q)
            return srv_fail(BPMF_E_INVALID, "request exceeds the slot size (max_nnz, max_q)");
    } else if (batch_bytes(1, nnz, nq, srv->m.S) > srv->capacity) {
        return srv_fail(BPMF_E_INVALID, "request exceeds one stream's memory budget");
    }
    Req r;
    r.id = id;
    r.cols.assign(h_cols, h_cols + nnz);
    r.vals.assign(h_vals, h_vals + nnz);
    r.qcols.assign(h_q_cols, h_q_cols + nq);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return srv_fail(BPMF_E_STATE, "server stopped: " + srv->error);
        r.t_submit = Clock::now();
        srv->queue.push_back(std::move(r));
        srv->submitted += 1;
    }
    srv->cv_submit.notify_one();
    return BPMF_OK;
}

bpmf_status bpmf_server_poll(bpmf_server *srv, int32_t max_results, int64_t *ids, int64_t *offsets,
                             float *h_preds, int64_t pred_capacity, double *latency_s, int32_t *n_out)
{
    if (!srv || !n_out) return srv_fail(BPMF_E_INVALID, "NULL argument");
    *n_out = 0;
    if (max_results <= 0) return BPMF_OK;
    std::lock_guard<std::mutex> lk(srv->mu);
    int64_t pos = 0;
    int32_t k = 0;
    if (offsets) offsets[0] = 0;
    while (k < max_results && !srv->done.empty()) {
        Done &d = srv->done.front();
        if (pos + (int64_t)d.preds.size() > pred_capacity) break;
        if (ids) ids[k] = d.id;
        if (h_preds) std::memcpy(h_preds + pos, d.preds.data(), 4 * d.preds.size());
        pos += (int64_t)d.preds.size();
        if (offsets) offsets[k + 1] = pos;
        if (latency_s) latency_s[k] = d.latency;
        srv->done.pop_front();
        ++k;
    }
    *n_out = k;
    if (!srv->error.empty()) return srv_fail(BPMF_E_HIP, srv->error);
    return BPMF_OK;
}

bpmf_status bpmf_server_drain(bpmf_server *srv)
{
    if (!srv) return srv_fail(BPMF_E_STATE, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->completed >= srv->submitted || !srv->error.empty(); });
    if (!srv->error.empty()) return srv_fail(BPMF_E_HIP, srv->error);
    return BPMF_OK;
}

bpmf_status bpmf_server_get_stats(bpmf_server *srv, bpmf_server_stats *st)
{
    if (!srv || !st) return srv_fail(BPMF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *st = srv->stats;
    return BPMF_OK;
}

bpmf_status bpmf_server_replay(bpmf_server *srv, int64_t n, const double *arrival_s, const int64_t *h_ptr,
                               const int32_t *h_cols, const float *h_vals, const int64_t *h_q_ptr,
                               const int32_t *h_q_cols, float *h_out, double *latency_s)
{
    if (!srv) return srv_fail(BPMF_E_STATE, "NULL server");
    if (n < 0 || (n > 0 && (!arrival_s || !h_ptr || !h_q_ptr || !h_out || !latency_s)))
        return srv_fail(BPMF_E_INVALID, "bad replay arguments");
    std::atomic<int> submit_err{0};
    std::string submit_msg;
    const auto t0 = Clock::now();
    std::thread client([&] {
        for (int64_t i = 0; i < n; ++i) {
            const auto due = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
            // sleep to ~100 us before the arrival, then spin
            const auto early = due - std::chrono::microseconds(100);
            if (Clock::now() < early) std::this_thread::sleep_until(early);
            while (Clock::now() < due) {
            }
            bpmf_status st = bpmf_server_submit(srv, i, (int32_t)(h_ptr[i + 1] - h_ptr[i]), h_cols + h_ptr[i],
                                                h_vals + h_ptr[i], (int32_t)(h_q_ptr[i + 1] - h_q_ptr[i]),
                                                h_q_cols + h_q_ptr[i]);
            if (st != BPMF_OK) {
                submit_err = (int)st;
                submit_msg = bpmf_last_error();
                return;
            }
        }
    });
    client.join();
    if (submit_err) return srv_fail((bpmf_status)submit_err.load(), submit_msg);
    bpmf_status st = bpmf_server_drain(srv);
    if (st != BPMF_OK) return st;
    // collect everything finished
    std::lock_guard<std::mutex> lk(srv->mu);
    while (!srv->done.empty()) {
        Done &d = srv->done.front();
        if (d.id >= 0 && d.id < n) {
            std::copy(d.preds.begin(), d.preds.end(), h_out + h_q_ptr[d.id]);
            latency_s[d.id] = d.latency;
        }
        srv->done.pop_front();
    }
    return BPMF_OK;
}

bpmf_status bpmf_server_destroy(bpmf_server *srv)
{
    if (!srv) return BPMF_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_submit.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    if (srv->r_stop) __atomic_store_n(srv->r_stop, 1, __ATOMIC_RELEASE);
    if (srv->r_fb_stream) {
        hipStreamSynchronize(srv->r_fb_stream);
        hipStreamDestroy(srv->r_fb_stream);
    }
    if (srv->r_stream) {
        hipStreamSynchronize(srv->r_stream);
        hipStreamDestroy(srv->r_stream);
    }
    if (srv->r_dev) hipFree(srv->r_dev);
    if (srv->r_slots) hipHostFree(srv->r_slots);
    if (srv->r_stop) hipHostFree(srv->r_stop);
    for (auto &sl : srv->slots) {
        if (sl.stream) hipStreamSynchronize(sl.stream);
        if (sl.done) hipEventDestroy(sl.done);
        if (sl.stream) hipStreamDestroy(sl.stream);
        if (sl.d_buf) hipFree(sl.d_buf);
        if (sl.h_buf) hipHostFree(sl.h_buf);
        if (sl.h_out) hipHostFree(sl.h_out);
    }
    delete srv;
    return BPMF_OK;
}

}  // extern "C"
