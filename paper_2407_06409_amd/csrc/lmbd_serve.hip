// Serving runtime: continuous batching of independent structures on one device.
//
// One device pool, carved into per-batch workspaces by a first-fit free list.
// Each slot is a host thread with its own lmbd context and HIP stream (default
// priority).  A free slot takes the longest prefix of the FIFO queue whose
// exact footprint fits in one free block and in the batch caps, and runs it as
// one lmbd_compute_batch call on host arrays; admission therefore follows the
// measured device footprint of the work, and batches of different slots run
// concurrently on the device.  A batch that fails is re-run request by request
// so that one bad structure does not fail its neighbours; results of a request
// do not depend on its batch (the kernels are batch-independent bitwise).
#include "lmbd.h"
#include "lmbd_host.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace lmbd;

namespace {

constexpr size_t kPoolAlign = 4096;

struct Request {
    uint64_t ticket = 0;
    lmbd_structure s{};
    StructCounts counts;
    lmbd_request_info info{};
};

}  // namespace

struct lmbd_server {
    lmbd_server_config cfg{};
    lmbd_params params{};
    std::vector<double> c_n, omega, weight;
    std::vector<lmbd_species> species;
    char* pool = nullptr;
    std::map<size_t, size_t> free_blocks;  // offset -> bytes, coalesced
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    std::vector<std::thread> slots;
    bool stop = false;
    uint64_t next_ticket = 1, next_batch = 1;
    int in_flight = 0;
    size_t pool_used = 0;
    lmbd_server_stats stats{};
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    size_t largest_free() const {
        size_t m = 0;
        for (const auto& b : free_blocks) m = std::max(m, b.second);
        return m;
    }

    // first fit; the caller has checked that a block is large enough
    size_t take(size_t bytes) {
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_blocks.erase(it);
            if (rest) free_blocks[off + bytes] = rest;
            pool_used += bytes;
            stats.pool_peak = std::max(stats.pool_peak, pool_used);
            return off;
        }
        return (size_t)-1;
    }

    void give_back(size_t off, size_t bytes) {
        pool_used -= bytes;
        auto it = free_blocks.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_blocks.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_blocks.erase(nx);
        }
        if (it != free_blocks.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_blocks.erase(it);
            }
        }
    }

    // Longest admissible prefix of the queue (lock held).  Empty when the head
    // does not fit in any free block yet.
    std::vector<Request*> form_batch(size_t& bytes) {
        std::vector<Request*> batch;
        std::vector<const StructCounts*> parts;
        const size_t room = largest_free();
        int64_t atoms = 0;
        bytes = 0;
        for (Request* r : queue) {
            if (!batch.empty()) {
                if (cfg.max_batch_requests > 0 && (int)batch.size() >= cfg.max_batch_requests) break;
                if (cfg.max_batch_atoms > 0 && atoms + r->s.n_atoms > cfg.max_batch_atoms) break;
            }
            parts.push_back(&r->counts);
            size_t b = 0;
            if (layout_bytes(&params, (int)species.size(), parts, &b) != LMBD_OK) b = (size_t)-1;
            b = (b + kPoolAlign - 1) / kPoolAlign * kPoolAlign;
            if (b > room) break;
            batch.push_back(r);
            bytes = b;
            atoms += r->s.n_atoms;
        }
        return batch;
    }

    void slot_main(int slot) {
        lmbd_context* ctx = nullptr;
        hipStream_t stream = nullptr;
        const bool ready = hipSetDevice(cfg.device) == hipSuccess && lmbd_create(cfg.device, &ctx) == LMBD_OK &&
                           hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
        for (;;) {
            std::vector<Request*> batch;
            size_t bytes = 0, off = 0;
            uint64_t id = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop) return true;
                    if (queue.empty()) return false;
                    batch = form_batch(bytes);
                    return !batch.empty();
                });
                if (stop) break;
                off = take(bytes);
                queue.erase(queue.begin(), queue.begin() + batch.size());
                id = next_batch++;
                stats.batches++;
                in_flight++;
                stats.max_concurrent = std::max(stats.max_concurrent, in_flight);
                const double ts = now();
                for (Request* r : batch) {
                    r->info.t_start = ts;
                    r->info.batch = id;
                    r->info.batch_requests = (int)batch.size();
                    r->info.slot = slot;
                }
            }
            std::vector<lmbd_status> result(batch.size(), LMBD_E_DEVICE);
            std::vector<std::string> detail(batch.size());
            if (ready) {
                set_workspace(ctx, pool + off, bytes);
                std::vector<lmbd_structure> desc;
                for (Request* r : batch) desc.push_back(r->s);
                lmbd_status st = lmbd_compute_batch(ctx, &params, (int)species.size(), species.data(),
                                                    (int)desc.size(), desc.data(), LMBD_HOST, stream);
                if (st == LMBD_OK || desc.size() == 1) {
                    std::fill(result.begin(), result.end(), st);
                    if (st != LMBD_OK) detail[0] = lmbd_last_error(ctx);
                } else {
                    for (size_t i = 0; i < desc.size(); ++i) {
                        result[i] = lmbd_compute(ctx, &params, (int)species.size(), species.data(), &desc[i],
                                                 LMBD_HOST, stream);
                        if (result[i] != LMBD_OK) detail[i] = lmbd_last_error(ctx);
                    }
                }
                set_workspace(ctx, nullptr, 0);
            } else {
                for (auto& d : detail) d = "slot could not create its context or stream";
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                give_back(off, bytes);
                in_flight--;
                const double te = now();
                for (size_t i = 0; i < batch.size(); ++i) {
                    Request* r = batch[i];
                    r->info.status = result[i];
                    std::snprintf(r->info.detail, sizeof(r->info.detail), "%s", detail[i].c_str());
                    r->info.t_end = te;
                    r->info.done = 1;
                    stats.completed++;
                }
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
        if (stream) (void)hipStreamDestroy(stream);
        lmbd_destroy(ctx);
    }
};

extern "C" {

lmbd_status lmbd_server_create(const lmbd_server_config* config, const lmbd_params* params, int32_t n_species,
                               const lmbd_species* species_table, lmbd_server** out) {
    if (!out) return LMBD_E_INVALID_ARG;
    *out = nullptr;
    if (!config || !params || !species_table || n_species < 1) return LMBD_E_INVALID_ARG;
    if (config->n_slots < 1 || config->n_slots > 16) return LMBD_E_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || config->device < 0 || config->device >= ndev)
        return LMBD_E_INVALID_ARG;
    if (params->n_max < 2 || params->n_freq < 1 || !params->omega || !params->weight) return LMBD_E_INVALID_ARG;
    for (int i = 0; i < n_species; ++i)
        if (!(species_table[i].alpha0 > 0) || !(species_table[i].c6 > 0) || !(species_table[i].r0 > 0))
            return LMBD_E_INVALID_ARG;
    std::unique_ptr<lmbd_server> s(new lmbd_server());
    s->cfg = *config;
    s->params = *params;
    s->omega.assign(params->omega, params->omega + params->n_freq);
    s->weight.assign(params->weight, params->weight + params->n_freq);
    s->params.omega = s->omega.data();
    s->params.weight = s->weight.data();
    if (params->c_n) {
        s->c_n.assign(params->c_n, params->c_n + params->n_max + 1);
        s->params.c_n = s->c_n.data();
    }
    s->species.assign(species_table, species_table + n_species);
    if (hipSetDevice(config->device) != hipSuccess) return LMBD_E_DEVICE;
    size_t bytes = config->memory_budget;
    if (bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return LMBD_E_DEVICE;
        bytes = free_b / 10 * 8;
    }
    bytes = bytes / kPoolAlign * kPoolAlign;
    if (bytes < kPoolAlign) return LMBD_E_INVALID_ARG;
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LMBD_E_OOM : LMBD_E_DEVICE;
    s->pool = static_cast<char*>(p);
    s->free_blocks[0] = bytes;
    s->stats.pool_bytes = bytes;
    s->t0 = std::chrono::steady_clock::now();
    lmbd_server* raw = s.release();
    for (int i = 0; i < config->n_slots; ++i) raw->slots.emplace_back([raw, i] { raw->slot_main(i); });
    *out = raw;
    return LMBD_OK;
}

void lmbd_server_destroy(lmbd_server* server) {
    if (!server) return;
    {
        std::lock_guard<std::mutex> lk(server->mu);
        server->stop = true;
        for (Request* r : server->queue) {
            r->info.status = LMBD_E_CANCELLED;
            r->info.done = 1;
        }
        server->queue.clear();
    }
    server->cv_work.notify_all();
    server->cv_done.notify_all();
    for (std::thread& t : server->slots) t.join();
    if (server->pool) {
        (void)hipSetDevice(server->cfg.device);
        (void)hipFree(server->pool);
    }
    delete server;
}

lmbd_status lmbd_submit(lmbd_server* server, const lmbd_structure* request, uint64_t* ticket) {
    if (!server || !request || !ticket) return LMBD_E_INVALID_ARG;
    std::unique_ptr<Request> r(new Request());
    r->s = *request;
    for (int64_t i = 0; request->species && i < request->n_atoms; ++i)
        if (request->species[i] >= (int32_t)server->species.size()) return LMBD_E_INVALID_ARG;
    lmbd_status st = analyse_structure(&server->params, r->s, r->counts);
    if (st != LMBD_OK) return st;
    size_t alone = 0;
    st = layout_bytes(&server->params, (int)server->species.size(), {&r->counts}, &alone);
    if (st != LMBD_OK) return st;
    r->info.footprint = alone;
    if ((alone + kPoolAlign - 1) / kPoolAlign * kPoolAlign > server->stats.pool_bytes) return LMBD_E_OOM_ADMISSION;
    {
        std::lock_guard<std::mutex> lk(server->mu);
        if (server->stop) return LMBD_E_CANCELLED;
        r->ticket = server->next_ticket++;
        r->info.t_submit = server->now();
        r->info.status = LMBD_OK;
        *ticket = r->ticket;
        server->queue.push_back(r.get());
        server->requests.emplace(r->ticket, std::move(r));
        server->stats.submitted++;
    }
    server->cv_work.notify_one();
    return LMBD_OK;
}

lmbd_status lmbd_poll(lmbd_server* server, uint64_t ticket, lmbd_request_info* info) {
    if (!server || !info) return LMBD_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(server->mu);
    auto it = server->requests.find(ticket);
    if (it == server->requests.end()) return LMBD_E_INVALID_ARG;
    *info = it->second->info;
    return LMBD_OK;
}

lmbd_status lmbd_wait(lmbd_server* server, uint64_t ticket, lmbd_request_info* info) {
    if (!server || !info) return LMBD_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(server->mu);
    auto it = server->requests.find(ticket);
    if (it == server->requests.end()) return LMBD_E_INVALID_ARG;
    Request* r = it->second.get();
    server->cv_done.wait(lk, [&] { return r->info.done != 0; });
    *info = r->info;
    return LMBD_OK;
}

lmbd_status lmbd_release(lmbd_server* server, uint64_t ticket) {
    if (!server) return LMBD_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(server->mu);
    auto it = server->requests.find(ticket);
    if (it == server->requests.end() || !it->second->info.done) return LMBD_E_INVALID_ARG;
    server->requests.erase(it);
    return LMBD_OK;
}

lmbd_status lmbd_server_get_stats(lmbd_server* server, lmbd_server_stats* stats) {
    if (!server || !stats) return LMBD_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(server->mu);
    *stats = server->stats;
    return LMBD_OK;
}

}  // extern "C"
