// Continuous-batching request server (pe_submit / pe_wait / pe_cancel).
//
// One scheduler thread per context.  Requests are admitted in arrival order while the sum of
// their HBM footprints (the transient workspace their screens need) fits the context's budget
// minus what scenes and other workspaces already hold.  Every scheduling round packs work
// items -- single incidences -- from ALL admitted requests, round-robin, into one shared launch
// batch (different scenes, screens, frequency sets and bounce limits side by side), up to a
// pixel budget; requests with other contrib/precision flags go into the next round.  Each
// slot's result depends only on its own slot (per-slot order-preserving compaction and
// fixed-order PO sums), so a request's field is bitwise the same alone or in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <thread>

#include "pe_runtime.h"

namespace pe {

struct Request {
    pe_ticket id = 0;
    pe_scene sc = nullptr;
    pe_solve_desc d{};
    std::vector<double> inc, obs, freq;
    pe_result res{};
    pe_stats acc{};
    uint64_t footprint = 0;
    int next = 0;       // next incidence to schedule
    int done = 0;       // incidences finished
    pe_status status = 1;  // 1 = pending
    bool admitted = false, cancel = false;
    std::chrono::steady_clock::time_point t0;
};

struct Server {
    pe_ctx ctx;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> pending;  // not yet admitted
    std::list<std::shared_ptr<Request>> active;    // admitted, unfinished
    std::map<pe_ticket, std::shared_ptr<Request>> all;
    pe_ticket next_id = 1;
    uint64_t active_bytes = 0;
    bool stop = false;
    std::thread th;
    hipStream_t st = nullptr;
    Workspace ws;
    // stats
    std::vector<double> lat_ms;
    double max_conc = 0, batches = 0, batch_reqs = 0;

    explicit Server(pe_ctx c) : ctx(c), ws(c) {
        HIPCHK(hipSetDevice(ctx->device));
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        th = std::thread([this] { loop(); });
    }
    ~Server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        if (th.joinable()) th.join();
        ws.release();
        if (st) (void)hipStreamDestroy(st);
    }

    void finish(const std::shared_ptr<Request>& r, pe_status s) {
        r->status = s;
        if (r->sc) {
            r->sc->refs--;  // the scene may be destroyed from here on
            r->sc = nullptr;
        }
        if (r->admitted) active_bytes -= r->footprint;
        r->admitted = false;
        if (s == PE_OK) {
            lat_ms.push_back(std::chrono::duration<double, std::milli>(
                                 std::chrono::steady_clock::now() - r->t0).count());
            if (r->res.stats) *r->res.stats = r->acc;
        }
        cv_done.notify_all();
    }

    // Bytes of free budget the server may still admit into.
    uint64_t free_budget() const {
        const uint64_t used = ctx->used.load();
        const uint64_t others = used > ws.bytes() ? used - ws.bytes() : 0;
        return ctx->budget > others ? ctx->budget - others : 0;
    }

    void admit() {
        while (!pending.empty()) {
            auto& r = pending.front();
            if (r->cancel) {
                finish(r, PE_ECANCELED);
                pending.pop_front();
                continue;
            }
            if (!active.empty() && active_bytes + r->footprint > free_budget()) break;
            r->admitted = true;
            active_bytes += r->footprint;
            active.push_back(r);
            pending.pop_front();
        }
        max_conc = std::max(max_conc, (double)active.size());
    }

    void loop() {
        (void)hipSetDevice(ctx->device);
        const uint64_t px_budget = [] {
            const char* e = std::getenv("PE_BATCH_PIXELS");
            return e ? std::strtoull(e, nullptr, 10) : (uint64_t)1 << 25;
        }();
        for (;;) {
            struct Item {
                std::shared_ptr<Request> r;
                int inc;
            };
            std::vector<Item> items;
            int contrib = 0, precision = 0, secondary = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
                if (stop) {
                    for (auto& r : pending) finish(r, PE_ECANCELED);
                    for (auto& r : active) finish(r, PE_ECANCELED);
                    pending.clear();
                    active.clear();
                    return;
                }
                admit();
                for (auto it = active.begin(); it != active.end();) {
                    if ((*it)->cancel) {
                        finish(*it, PE_ECANCELED);
                        it = active.erase(it);
                    } else {
                        ++it;
                    }
                }
                if (active.empty()) continue;
                // round-robin over admitted requests sharing the first one's flags
                contrib = active.front()->d.contrib;
                precision = active.front()->d.precision;
                secondary = active.front()->d.secondary;
                uint64_t px = 0;
                bool progress = true;
                while (progress && (int)items.size() < kMaxSlots) {
                    progress = false;
                    for (auto& r : active) {
                        if (r->d.contrib != contrib || r->d.precision != precision ||
                            r->d.secondary != secondary)
                            continue;
                        if (r->next >= r->d.n_inc) continue;
                        const uint64_t p = (uint64_t)r->d.screen_w * r->d.screen_h;
                        if (!items.empty() && px + p > px_budget) continue;
                        items.push_back({r, r->next++});
                        px += p;
                        progress = true;
                        if ((int)items.size() >= kMaxSlots) break;
                    }
                    if (px >= px_budget) break;
                }
            }
            if (items.empty()) continue;
            // build slots (requests cannot vanish: they hold shared pointers)
            std::vector<SlotSpec> slots;
            for (auto& it : items) {
                auto v = make_slots(it.r->sc, &it.r->d, it.inc, 1);
                slots.push_back(v[0]);
            }
            uint64_t tot = 0;
            std::vector<uint64_t> base;
            for (auto& it : items) {
                base.push_back(tot);
                tot += (uint64_t)(it.r->d.obs_dir ? it.r->d.n_obs : 1) * it.r->d.n_freq * 4;
            }
            std::vector<double> E(tot * 2), R(tot);
            pe_stats acc{};
            pe_status s = PE_OK;
            std::string err;
            try {
                std::lock_guard<std::mutex> dev(ctx->mu);
                run_field_batch(ws, st, slots, contrib, precision, E.data(), R.data(), &acc,
                                secondary);
                HIPCHK(hipStreamSynchronize(st));
            } catch (const Error& e) {
                s = e.status;
                err = e.msg;
            } catch (const std::exception& e) {
                s = PE_EDEVICE;
                err = e.what();
            }
            std::lock_guard<std::mutex> lk(mu);
            batches += 1;
            {
                std::vector<Request*> uniq;
                for (auto& it : items)
                    if (std::find(uniq.begin(), uniq.end(), it.r.get()) == uniq.end()) uniq.push_back(it.r.get());
                batch_reqs += (double)uniq.size();
            }
            for (size_t i = 0; i < items.size(); i++) {
                auto& r = items[i].r;
                if (r->status != 1) continue;
                if (s != PE_OK) {
                    active.remove(r);
                    finish(r, s);
                    continue;
                }
                const uint64_t per = (uint64_t)(r->d.obs_dir ? r->d.n_obs : 1) * r->d.n_freq * 4;
                std::memcpy(r->res.E + (uint64_t)items[i].inc * per * 2, E.data() + base[i] * 2,
                            sizeof(double) * per * 2);
                if (r->res.rcs_dbsm)
                    std::memcpy(r->res.rcs_dbsm + (uint64_t)items[i].inc * per, R.data() + base[i],
                                sizeof(double) * per);
                r->done++;
            }
            // per-request statistics: share the batch counters by slot count
            for (size_t i = 0; i < items.size(); i++) {
                auto& r = items[i].r;
                const double f = 1.0 / (double)items.size();
                r->acc.ray_queries += acc.ray_queries * f;
                r->acc.exit_records += acc.exit_records * f;
                r->acc.po_terms += acc.po_terms * f;
                r->acc.march_rays += acc.march_rays * f;
                r->acc.march_hits += acc.march_hits * f;
                r->acc.march_cap_hits += acc.march_cap_hits * f;
            }
            for (auto it = active.begin(); it != active.end();) {
                auto& r = *it;
                if (r->status == 1 && r->done == r->d.n_inc) {
                    r->acc.time_ms = std::chrono::duration<double, std::milli>(
                                         std::chrono::steady_clock::now() - r->t0).count();
                    finish(r, PE_OK);
                    it = active.erase(it);
                } else {
                    ++it;
                }
            }
        }
    }
};

// Transient device bytes one request's batches need per incidence slot (ray state, lists,
// keys, records, PO partials), times the slots it can occupy at once.
static uint64_t request_footprint(const pe_solve_desc* d) {
    const uint64_t px = (uint64_t)d->screen_w * d->screen_h;
    const uint64_t per_px = batch_bytes_per_pixel(d);
    const uint64_t slots = std::min<uint64_t>(d->n_inc, std::max<uint64_t>(1, ((uint64_t)1 << 25) / px));
    return (slots * px * per_px + (64ull << 20)) / 8 * 9;
}

void server_shutdown(pe_ctx ctx) {
    Server* s = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->server_mu);
        s = ctx->server;
        ctx->server = nullptr;
    }
    delete s;
}

static Server* get_server(pe_ctx ctx) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) ctx->server = new Server(ctx);
    return ctx->server;
}

}  // namespace pe

using namespace pe;

extern "C" {

pe_status pe_submit(pe_ctx ctx, pe_scene scene, const pe_solve_desc* desc, pe_result* res,
                    pe_ticket* ticket) {
    API_BEGIN
    if (!ctx || !res || !res->E || !ticket) return set_error(PE_EINVAL, "null argument");
    validate_solve(scene, desc);
    if (scene->ctx != ctx) return set_error(PE_EINVAL, "scene belongs to another context");
    if (desc->geometry != PE_GEOM_PLAIN)
        return set_error(PE_EUNSUPPORTED, "the server batches plain-geometry solves");
    auto r = std::make_shared<Request>();
    r->sc = scene;
    r->d = *desc;
    r->inc.assign(desc->inc_dir, desc->inc_dir + 3 * desc->n_inc);
    r->d.inc_dir = r->inc.data();
    if (desc->obs_dir) {
        r->obs.assign(desc->obs_dir, desc->obs_dir + 3 * desc->n_obs);
        r->d.obs_dir = r->obs.data();
    }
    r->freq.assign(desc->freq_hz, desc->freq_hz + desc->n_freq);
    r->d.freq_hz = r->freq.data();
    r->res = *res;
    r->footprint = request_footprint(desc);
    if (r->footprint > ctx->budget) return set_error(PE_ENOMEM, "request footprint exceeds the context budget");
    r->t0 = std::chrono::steady_clock::now();
    Server* s = get_server(ctx);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        scene->refs++;  // released by Server::finish
        r->id = s->next_id++;
        s->all[r->id] = r;
        s->pending.push_back(r);
        *ticket = r->id;
    }
    s->cv_work.notify_all();
    return PE_OK;
    API_END
}

pe_status pe_request_footprint(const pe_solve_desc* desc, uint64_t* bytes) {
    API_BEGIN
    if (!desc || !bytes) return set_error(PE_EINVAL, "null argument");
    validate_solve(nullptr, desc, false);
    *bytes = request_footprint(desc);
    return PE_OK;
    API_END
}

pe_status pe_wait(pe_ctx ctx, pe_ticket ticket, int64_t timeout_us) {
    API_BEGIN
    if (!ctx) return set_error(PE_EINVAL, "null context");
    Server* s = get_server(ctx);
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(PE_EINVAL, "unknown ticket");
    auto r = it->second;
    auto ready = [&] { return r->status != 1; };
    if (timeout_us < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return PE_ETIMEOUT;
    }
    const pe_status st = r->status;
    s->all.erase(ticket);
    if (st != PE_OK) return set_error(st, st == PE_ECANCELED ? "request cancelled" : "request failed");
    return PE_OK;
    API_END
}

pe_status pe_cancel(pe_ctx ctx, pe_ticket ticket) {
    API_BEGIN
    if (!ctx) return set_error(PE_EINVAL, "null context");
    Server* s = get_server(ctx);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return set_error(PE_EINVAL, "unknown ticket");
        it->second->cancel = true;
    }
    s->cv_work.notify_all();
    return PE_OK;
    API_END
}

pe_status pe_server_stats(pe_ctx ctx, double out[6], int32_t reset) {
    API_BEGIN
    if (!ctx || !out) return set_error(PE_EINVAL, "null argument");
    Server* s = get_server(ctx);
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
        if (v.empty()) return 0.0;
        const size_t i = std::min(v.size() - 1, (size_t)std::ceil(q * v.size()) - (q > 0 ? 1 : 0));
        return v[i];
    };
    double mean = 0;
    for (double x : v) mean += x;
    out[0] = (double)v.size();
    out[1] = pct(0.5);
    out[2] = pct(0.99);
    out[3] = v.empty() ? 0.0 : mean / v.size();
    out[4] = s->max_conc;
    out[5] = s->batches > 0 ? s->batch_reqs / s->batches : 0.0;
    if (reset) {
        s->lat_ms.clear();
        s->max_conc = (double)s->active.size();
        s->batches = s->batch_reqs = 0;
    }
    return PE_OK;
    API_END
}

}  // extern "C"
