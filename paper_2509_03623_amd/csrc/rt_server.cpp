// rt_server.cpp -- continuous-batching render server on one GPU.
//
// rt_submit validates a request on the host, deep-copies its problem and
// queues it.  A scheduler thread
//   1. retires finished launches (event queries) and frees their budget/slots,
//   2. admits queued requests in arrival order while their HBM footprint fits
//      the budget and a slot is free,
//   3. starts admitted work on an idle stream: the admitted plain forward
//      requests that are too small to fill the device alone go into one
//      persistent launch whose workgroups pull (request, tile, channel block)
//      items from a device counter; the admitted gradient requests (forward,
//      fused L2 loss + cotangent, adjoint) that are too small to fill the
//      device alone go into one batched sequence of persistent launches
//      (tape, reverse march, chain; rt_serve_grad.hip); a request that fills
//      the device alone (the direct renderer's launch shape) or one with the
//      neural CO layer runs on a stream of its own.
// Requests that arrive while launches run are admitted as budget and slots
// free up and start on the next idle stream, so their work overlaps on the
// device with what is already running.  A forward cube depends only on its
// own request (each ray is marched by one lane with the same code whatever
// else is in the batch); a gradient request's routing depends only on its
// own shape, and its result on the rest of its batch only through the order
// of the accumulators' atomic additions.  Device memory: the budget covers
// the footprints of admitted requests plus the library scratch that idle
// streams keep for their next launch (reusing it saves a fresh mapping per
// launch); when a request does not fit, the idle streams' scratch is released
// first.  A launch whose scratch allocation fails while other launches run
// (memory held outside the server's account) puts its batch back at the head
// of the admitted queue and starts nothing until a running launch ends; the
// idle streams then give their scratch back before the next start.  With
// nothing running, the memory pool is trimmed back to the device and the
// batch tries once more before it fails.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "rt_adjoint.h"
#include "rt_host.h"
#include "rt_serve.h"

using namespace rt;

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t id = 0;
    rt_request rq{};
    std::vector<double> lev_e, lev_g, vk;
    rt_mlp mlp{};
    int state = RT_TICKET_QUEUED;
    int status = RT_PENDING;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    double loss = 0.0;
    uint64_t footprint = 0, ray_samples = 0;
    bool own_stream = false;   // large or neural request
    bool grad_batch = false;   // small gradient request (batched launches)
    bool trimmed = false;      // retried once after the memory pool was trimmed
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<Req *> reqs;
    ServeDesc *d_desc = nullptr, *h_desc = nullptr;
    float *d_vch = nullptr, *h_vch = nullptr;
    size_t vch_cap = 0;
    uint32_t *d_counter = nullptr;
    double *d_loss = nullptr, *h_loss = nullptr;
    GradDesc *d_gdesc = nullptr, *h_gdesc = nullptr;
    uint32_t *d_gcount = nullptr;   // item counters of the three batched gradient passes
    uint64_t retained = 0;          // scratch the idle stream keeps (charged to the budget)
    uint64_t excess = 0;            // that scratch, charged to the running launch
};

__global__ void zero_u32(uint32_t *p) { *p = 0u; }

} // namespace

struct rt_server {
    rt_server_cfg cfg{};
    int ncu = 0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_id = 1;
    std::map<uint64_t, std::unique_ptr<Req>> tickets;
    std::deque<Req *> pending, admitted;
    uint64_t budget_used = 0;      // footprints of admitted requests, plus scratch held by running launches
    uint64_t retained_idle = 0;    // scratch held by idle streams
    bool hold = false;             // a launch ran out of device memory: start nothing until a lane retires
    bool squeeze = false;          // ... and then release the idle streams' scratch before the next start
    int slots_used = 0;
    std::vector<Lane> lanes;
};

namespace {

// Device memory a request occupies while it runs: its inputs and outputs and
// the library's scratch, each stream workspace counted at the size it
// actually holds (workspace_round).
uint64_t footprint(const rt_request &r, bool grad_batched) {
    const rt_problem &p = r.problem;
    const uint64_t nn = (uint64_t)p.grid.nr * p.grid.nz, nr = p.grid.nr;
    const uint64_t npix = (uint64_t)p.cam.nx * p.cam.ny, cube = 4ull * p.spec.nch * npix;
    const uint64_t M = npix * p.nsamp;
    uint64_t b = 4 * (3 * nn + 2 * nr) + cube;
    if (p.mlp) b += 4ull * RT_MLP_PARAMS + 16 * M + (1u << 20);
    if (r.kind == RT_REQ_FWD_LOSS) b += cube;   // target
    if (r.kind == RT_REQ_FWD_LOSS && r.beam.bmaj_px > 0.0) {
        // convolved cube and the beam's weights (stream workspaces)
        const double sig = r.beam.bmaj_px / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        const uint64_t side = 2 * (uint64_t)std::ceil(3.0 * sig) + 1;
        b += workspace_round(cube) + workspace_round(4 * side * side);
    }
    if (r.kind == RT_REQ_FWD_ADJ && !p.mlp && grad_batched) {
        // target, grads, and the batched passes' tape, rays, cotangents,
        // accumulators (one workspace for the whole batch: rounding each
        // request's share up bounds it)
        b += cube + 4 * (3 * nn + 2 * nr);
        b += workspace_round(grad_batch_scratch_bytes(p.spec.nch, (long)npix, p.nsamp, p.grid.nr, p.grid.nz));
    } else if (r.kind == RT_REQ_FWD_ADJ) {
        const int ch = std::min(p.spec.nch, kLaunchChannels);
        b += cube + 4 * (3 * nn + 2 * nr) + workspace_round(8 * (3 * nn + 2 * nr));   // target, grads, accumulators
        // tape, rays, checkpoints, cotangents of one band of rows (gradient
        // requests run the fused L2 adjoint, which forms the cube)
        const uint64_t row = adjoint_bytes_per_pixel(ch, (long)npix, p.nsamp, true) * (uint64_t)p.cam.nx;
        b += workspace_round(std::min<uint64_t>(row * p.cam.ny,
                                                std::max<uint64_t>(row, adjoint_scratch_cap() / row * row)));
        if (p.mlp) b += 16 * M + 4ull * RT_MLP_PARAMS;
    }
    return b;
}

void finish(rt_server *sv, Req *r, int status) {
    r->status = status;
    r->state = status == RT_OK ? RT_TICKET_DONE : RT_TICKET_FAILED;
    r->t_done = now_ns();
    sv->budget_used -= r->footprint;
    sv->slots_used -= 1;
}

// a lane's launch is over: its charged scratch leaves the running total and
// what its stream now keeps is charged as idle
void lane_retired(rt_server *sv, Lane &L) {
    sv->budget_used -= L.excess;
    L.excess = 0;
    L.retained = stream_workspace_bytes(L.st);
    sv->retained_idle += L.retained;
}

rt_status lane_vch_capacity(Lane &L, size_t n) {
    if (n <= L.vch_cap) return RT_OK;
    if (L.d_vch) (void)hipFree(L.d_vch);
    if (L.h_vch) (void)hipHostFree(L.h_vch);
    L.d_vch = nullptr;
    L.h_vch = nullptr;
    L.vch_cap = 0;
    hipError_t e = hipMalloc(&L.d_vch, n * sizeof(float));
    if (e == hipSuccess) e = hipHostMalloc(&L.h_vch, n * sizeof(float), hipHostMallocDefault);
    if (e != hipSuccess) return fail_hip(e, "server channel buffers");
    L.vch_cap = n;
    return RT_OK;
}

// one persistent launch over every request of the batch
rt_status launch_batch(rt_server *sv, Lane &L, std::vector<Req *> &batch) {
    size_t nv = 0;
    for (Req *r : batch) nv += (size_t)(r->rq.problem.spec.nch + 15) / 16 * 16;
    rt_status rs = lane_vch_capacity(L, nv);
    if (rs != RT_OK) return rs;
    uint32_t items = 0;
    size_t vo = 0, max_n = 0;
    bool with_loss = false;
    for (size_t i = 0; i < batch.size(); ++i) {
        const rt_problem &p = batch[i]->rq.problem;
        ServeDesc &D = L.h_desc[i];
        std::memset(&D, 0, sizeof D);
        rs = build_launch(&p, &D.g, &D.s);
        if (rs != RT_OK) return rs;
        const int nch = p.spec.nch, padded = (nch + 15) / 16 * 16;
        for (int c = 0; c < padded; ++c) L.h_vch[vo + c] = c < nch ? (float)p.spec.v_kms[c] : 0.0f;
        D.vch = L.d_vch + vo;
        vo += padded;
        D.cube = batch[i]->rq.cube;
        D.nch = nch;
        D.nblk = padded / 16;
        D.tiles_x = (p.cam.nx + kServeTile - 1) / kServeTile;
        D.item0 = items;
        if (batch[i]->rq.kind == RT_REQ_FWD_LOSS) {
            D.target = batch[i]->rq.target;
            D.loss = L.d_loss + i;
            with_loss = true;
            max_n = std::max(max_n, (size_t)nch * p.cam.nx * p.cam.ny);
        }
        items += (uint32_t)(D.tiles_x * ((p.cam.ny + kServeTile - 1) / kServeTile) * D.nblk);
    }
    hipError_t e = hipMemcpyAsync(L.d_desc, L.h_desc, sizeof(ServeDesc) * batch.size(), hipMemcpyHostToDevice, L.st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.d_vch, L.h_vch, sizeof(float) * vo, hipMemcpyHostToDevice, L.st);
    if (e != hipSuccess) return fail_hip(e, "server upload");
    hipLaunchKernelGGL(zero_u32, dim3(1), dim3(1), 0, L.st, L.d_counter);
    if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e, "server counter");
    e = launch_serve_fwd(L.d_desc, (int)batch.size(), items, L.d_counter, sv->ncu * kServeWorkgroupsPerCU, L.st);
    if (e != hipSuccess) return fail_hip(e, "server batch launch");
    for (Req *r : batch) {
        const rt_request &q = r->rq;
        if (q.kind != RT_REQ_FWD_LOSS || !(q.beam.bmaj_px > 0.0)) continue;
        rs = beam_in_place(q.cube, q.problem.spec.nch, q.problem.cam.ny, q.problem.cam.nx, q.beam, L.st);
        if (rs != RT_OK) return rs;
    }
    if (with_loss) {
        e = launch_l2_batch(L.d_desc, (int)batch.size(), L.d_loss, max_n, L.st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(L.h_loss, L.d_loss, sizeof(double) * batch.size(), hipMemcpyDeviceToHost, L.st);
        if (e != hipSuccess) return fail_hip(e, "server batch loss");
    }
    return RT_OK;
}

// one batched sequence of gradient launches over every request of the batch
rt_status launch_grad(rt_server *sv, Lane &L, std::vector<Req *> &batch) {
    constexpr int kPad = kGradSlice;
    size_t nv = 0, scratch = 0;
    for (Req *r : batch) {
        const rt_problem &p = r->rq.problem;
        nv += (size_t)(p.spec.nch + kPad - 1) / kPad * kPad;
        scratch += grad_batch_scratch_bytes(p.spec.nch, (long)p.cam.nx * p.cam.ny, p.nsamp, p.grid.nr, p.grid.nz);
    }
    rt_status rs = lane_vch_capacity(L, nv);
    if (rs != RT_OK) return rs;
    hipError_t e;
    char *base = (char *)stream_workspace(L.st, kWsGradBatch, scratch, &e);
    if (!base) return fail_hip(e, "batched gradient scratch");
    uint32_t items[3] = {0, 0, 0};
    size_t vo = 0;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    for (size_t i = 0; i < batch.size(); ++i) {
        const rt_request &q = batch[i]->rq;
        const rt_problem &p = q.problem;
        GradDesc &D = L.h_gdesc[i];
        std::memset(&D, 0, sizeof D);
        rs = build_launch(&p, &D.g, &D.s);
        if (rs != RT_OK) return rs;
        const int nch = p.spec.nch, padded = (nch + kPad - 1) / kPad * kPad;
        for (int c = 0; c < padded; ++c) L.h_vch[vo + c] = c < nch ? (float)p.spec.v_kms[c] : 0.0f;
        D.vch = L.d_vch + vo;
        vo += padded;
        const size_t npix = (size_t)p.cam.nx * p.cam.ny, ns = p.nsamp;
        D.nch = nch;
        D.nblk = padded / kPad;
        double shift = 0.0;
        (void)group_shift(p.spec.v_kms, nch, kGradLanes, kGradLaneCB, &shift);   // checked at submission
        D.vshift = (float)shift;
        D.target = q.target;
        D.cube = q.cube;
        D.tape = (float4 *)base;
        base += al(sizeof(float4) * ns * npix);
        D.rays = (float4 *)base;
        base += al(sizeof(float4) * npix);
        D.cot = (float4 *)base;
        base += al(sizeof(float4) * D.nblk * ns * npix);
        D.span = (int2 *)base;
        base += al(sizeof(int2) * npix);
        D.acc = (double *)base;
        base += al(sizeof(double) * (3 * (size_t)p.grid.nr * p.grid.nz + 2 * (size_t)p.grid.nr));
        D.out[0] = q.grads.d_ln_nh2;
        D.out[1] = q.grads.d_temp_k;
        D.out[2] = q.grads.d_vphi_kms;
        D.out[3] = q.grads.d_z_lo_au;
        D.out[4] = q.grads.d_z_up_au;
        D.loss = L.d_loss + i;
        // chain field passes: each requested field; the first also takes the surfaces
        D.nfp = 0;
        for (int f = 0; f < 3; ++f)
            if (D.out[f]) D.fields[D.nfp++] = f;
        if (D.nfp == 0) D.fields[D.nfp++] = 3;
        uint32_t n[3];
        grad_batch_items(nch, (long)npix, p.nsamp, D.nfp, n, &D.chunks);
        for (int k = 0; k < 3; ++k) {
            D.item0[k] = items[k];
            items[k] += n[k];
        }
    }
    e = hipMemcpyAsync(L.d_gdesc, L.h_gdesc, sizeof(GradDesc) * batch.size(), hipMemcpyHostToDevice, L.st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.d_vch, L.h_vch, sizeof(float) * vo, hipMemcpyHostToDevice, L.st);
    if (e != hipSuccess) return fail_hip(e, "server gradient upload");
    e = launch_grad_batch(L.d_gdesc, L.h_gdesc, (int)batch.size(), items, L.d_gcount,
                          sv->ncu * kServeWorkgroupsPerCU, L.st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(L.h_loss, L.d_loss, sizeof(double) * batch.size(), hipMemcpyDeviceToHost, L.st);
    return e == hipSuccess ? RT_OK : fail_hip(e, "server gradient batch");
}

// a request on a stream of its own: a large or neural forward, or the fused
// forward + L2 loss + adjoint (the reverse march forms dL/dI = 2 (I - D) from
// its own forward sweep and writes the cube)
rt_status launch_single(Lane &L, Req *r) {
    const rt_request &q = r->rq;
    const rt_problem *p = &q.problem;
    rt_status rs;
    if (q.kind == RT_REQ_FWD_ADJ) {
        rs = p->mlp ? adjoint_mlp(p, nullptr, &q.grads, q.cube, L.st, q.target)
                    : adjoint_grid(p, nullptr, &q.grads, q.cube, L.st, q.target);
        if (rs != RT_OK) return rs;
        const size_t n = (size_t)p->spec.nch * p->cam.nx * p->cam.ny;
        hipError_t e = launch_l2_value(q.cube, q.target, n, L.d_loss, L.st);
        if (e == hipSuccess) e = hipMemcpyAsync(L.h_loss, L.d_loss, sizeof(double), hipMemcpyDeviceToHost, L.st);
        if (e != hipSuccess) return fail_hip(e, "loss");
        return RT_OK;
    }
    if (p->mlp) {
        rs = render_cube_mlp(p, q.cube, L.st);
    } else {
        Geometry g;
        Shade s;
        rs = build_launch(p, &g, &s);
        if (rs == RT_OK) rs = march_cube(p, g, s, q.cube, L.st);
    }
    if (rs != RT_OK || q.kind != RT_REQ_FWD_LOSS) return rs;
    if (q.beam.bmaj_px > 0.0) {
        rs = beam_in_place(q.cube, p->spec.nch, p->cam.ny, p->cam.nx, q.beam, L.st);
        if (rs != RT_OK) return rs;
    }
    const size_t n = (size_t)p->spec.nch * p->cam.nx * p->cam.ny;
    hipError_t e = launch_l2_value(q.cube, q.target, n, L.d_loss, L.st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.h_loss, L.d_loss, sizeof(double), hipMemcpyDeviceToHost, L.st);
    return e == hipSuccess ? RT_OK : fail_hip(e, "loss");
}

void scheduler(rt_server *sv) {
    (void)hipSetDevice(sv->cfg.device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        bool progress = false;
        // 1. retire finished launches
        for (Lane &L : sv->lanes) {
            if (!L.busy) continue;
            const hipError_t q = hipEventQuery(L.ev);
            if (q == hipErrorNotReady) continue;
            for (size_t i = 0; i < L.reqs.size(); ++i) {
                Req *r = L.reqs[i];
                if (r->rq.kind != RT_REQ_FWD) r->loss = L.h_loss[i];
                finish(sv, r, q == hipSuccess ? RT_OK : RT_EDEVICE);
            }
            lane_retired(sv, L);
            L.reqs.clear();
            L.busy = false;
            sv->hold = false;
            progress = true;
        }
        // 2. admission in arrival order, by footprint and slots
        while (!sv->pending.empty()) {
            Req *r = sv->pending.front();
            if (sv->slots_used >= sv->cfg.max_slots) break;
            auto fits = [&] { return sv->budget_used + sv->retained_idle + r->footprint <= sv->cfg.hbm_budget_bytes; };
            if (!fits() && sv->retained_idle > 0) {
                // make room: the idle streams give their scratch back
                for (Lane &L : sv->lanes) {
                    if (L.busy || L.retained == 0) continue;
                    release_stream_workspaces(L.st);
                    sv->retained_idle -= L.retained;
                    L.retained = 0;
                }
            }
            if (!fits()) break;
            sv->pending.pop_front();
            sv->budget_used += r->footprint;
            sv->slots_used += 1;
            r->state = RT_TICKET_RUNNING;
            r->t_admit = now_ns();
            sv->admitted.push_back(r);
            progress = true;
        }
        // 3. start admitted work on idle streams
        if (sv->squeeze && !sv->hold) {
            // (the frees complete before the next allocation, so the memory
            // pool can hand their blocks to any stream)
            for (Lane &L : sv->lanes) {
                if (L.busy || L.retained == 0) continue;
                release_stream_workspaces(L.st);
                (void)hipStreamSynchronize(L.st);
                sv->retained_idle -= L.retained;
                L.retained = 0;
            }
            sv->squeeze = false;
        }
        for (Lane &L : sv->lanes) {
            if (L.busy || sv->admitted.empty() || sv->hold) continue;
            std::vector<Req *> batch;
            if (sv->admitted.front()->own_stream) {
                batch.push_back(sv->admitted.front());
                sv->admitted.pop_front();
            } else {
                // every admitted request of the front one's kind of batch
                const bool grad = sv->admitted.front()->grad_batch;
                for (auto it = sv->admitted.begin(); it != sv->admitted.end();) {
                    if (!(*it)->own_stream && (*it)->grad_batch == grad && (int)batch.size() < sv->cfg.max_slots) {
                        batch.push_back(*it);
                        it = sv->admitted.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            // the scratch this stream keeps is now the running launch's
            sv->retained_idle -= L.retained;
            L.excess = L.retained;
            L.retained = 0;
            sv->budget_used += L.excess;
            // launch without holding the lock, so submissions are not held up
            // (the batch and the lane belong to this thread until then)
            lk.unlock();
            Req *front = batch.front();
            rt_status rs = front->own_stream ? launch_single(L, front)
                         : front->grad_batch ? launch_grad(sv, L, batch) : launch_batch(sv, L, batch);
            hipError_t e = hipSuccess;
            if (rs == RT_OK) e = hipEventRecord(L.ev, L.st);
            lk.lock();
            if (rs != RT_OK || e != hipSuccess) {
                // the stream may hold partial work: wait for it and give its scratch back
                (void)hipStreamSynchronize(L.st);
                release_stream_workspaces(L.st);
                bool running = false, trimmed = false;
                for (const Lane &O : sv->lanes) running = running || O.busy;
                for (const Req *r : batch) trimmed = trimmed || r->trimmed;
                if (rs == RT_ENOMEM && running) {
                    // device memory is short of what the budget assumed (memory
                    // held outside the server): the batch goes back to the head
                    // of the admitted queue, still charged, and waits for a
                    // running launch to end and return its memory
                    for (auto it = batch.rbegin(); it != batch.rend(); ++it) sv->admitted.push_front(*it);
                    sv->hold = true;
                    sv->squeeze = true;
                } else if (rs == RT_ENOMEM && !trimmed) {
                    // nothing left to wait for: the idle streams' scratch and
                    // the memory pool's free blocks (which another stream may
                    // not be allowed to reuse) go back to the device, and the
                    // batch tries once more
                    for (Lane &O : sv->lanes) {
                        if (O.retained == 0) continue;
                        release_stream_workspaces(O.st);
                        (void)hipStreamSynchronize(O.st);
                        sv->retained_idle -= O.retained;
                        O.retained = 0;
                    }
                    trim_memory_pool();
                    for (Req *r : batch) r->trimmed = true;
                    for (auto it = batch.rbegin(); it != batch.rend(); ++it) sv->admitted.push_front(*it);
                } else {
                    for (Req *r : batch) finish(sv, r, rs != RT_OK ? rs : RT_EDEVICE);
                }
                lane_retired(sv, L);
                continue;
            }
            L.reqs = batch;
            L.busy = true;
            progress = true;
        }
        if (progress) sv->cv.notify_all();
        bool idle = sv->pending.empty() && sv->admitted.empty();
        for (Lane &L : sv->lanes) idle = idle && !L.busy;
        if (sv->stop && idle) break;
        if (!progress) sv->cv.wait_for(lk, std::chrono::microseconds(idle ? 2000 : 50));
    }
}

} // namespace

extern "C" {

rt_status rt_server_create(const rt_server_cfg *cfg, rt_server **out) {
    if (!cfg || !out) return fail(RT_EINVAL, "NULL argument");
    if (cfg->max_slots < 1 || cfg->max_slots > 1024) return fail(RT_EINVAL, "max_slots must be 1..1024");
    if (cfg->max_pending < 1) return fail(RT_EINVAL, "max_pending must be >= 1");
    if (cfg->streams < 1 || cfg->streams > 8) return fail(RT_EINVAL, "streams must be 1..8");
    if (cfg->hbm_budget_bytes == 0) return fail(RT_EINVAL, "hbm_budget_bytes must be > 0");
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
    std::unique_ptr<rt_server> sv(new rt_server);
    sv->cfg = *cfg;
    e = hipDeviceGetAttribute(&sv->ncu, hipDeviceAttributeMultiprocessorCount, cfg->device);
    if (e != hipSuccess) return fail_hip(e, "device query");
    sv->lanes.resize(cfg->streams);
    for (Lane &L : sv->lanes) {
        if ((e = hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&L.ev, hipEventDisableTiming)) != hipSuccess ||
            (e = hipMalloc(&L.d_desc, sizeof(ServeDesc) * cfg->max_slots)) != hipSuccess ||
            (e = hipHostMalloc(&L.h_desc, sizeof(ServeDesc) * cfg->max_slots, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&L.d_counter, sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&L.d_loss, sizeof(double) * cfg->max_slots)) != hipSuccess ||
            (e = hipHostMalloc(&L.h_loss, sizeof(double) * cfg->max_slots, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&L.d_gdesc, sizeof(GradDesc) * cfg->max_slots)) != hipSuccess ||
            (e = hipHostMalloc(&L.h_gdesc, sizeof(GradDesc) * cfg->max_slots, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&L.d_gcount, 3 * sizeof(uint32_t))) != hipSuccess) {
            rt_status st = fail_hip(e, "server resources");
            rt_server_destroy(sv.release());
            return st;
        }
        for (int i = 0; i < cfg->max_slots; ++i) L.h_loss[i] = 0.0;
        // channel velocities of a full batch of up to kLaunchChannels-channel requests
        rt_status rs = lane_vch_capacity(L, (size_t)cfg->max_slots * kLaunchChannels);
        if (rs != RT_OK) {
            rt_server_destroy(sv.release());
            return rs;
        }
    }
    rt_server *p = sv.release();
    p->th = std::thread(scheduler, p);
    *out = p;
    return RT_OK;
}

rt_status rt_submit(rt_server *sv, const rt_request *rq, uint64_t *ticket) {
    if (!sv || !rq || !ticket) return fail(RT_EINVAL, "NULL argument");
    rt_status st = validate(&rq->problem);
    if (st != RT_OK) return st;
    if (rq->kind != RT_REQ_FWD && rq->kind != RT_REQ_FWD_ADJ && rq->kind != RT_REQ_FWD_LOSS)
        return fail(RT_EINVAL, "unknown request kind");
    if (!rq->cube) return fail(RT_EINVAL, "cube is NULL");
    if (rq->kind == RT_REQ_FWD_LOSS && !rq->target) return fail(RT_EINVAL, "target is NULL");
    const rt_beam &bm = rq->beam;
    if (bm.bmaj_px != 0.0 || bm.bmin_px != 0.0 || bm.bpa_deg != 0.0) {
        if (rq->kind != RT_REQ_FWD_LOSS) return fail(RT_EINVAL, "a beam applies to RT_REQ_FWD_LOSS requests only");
        rt_status bs = validate_beam(bm);
        if (bs != RT_OK) return bs;
    }
    if (rq->kind == RT_REQ_FWD_ADJ) {
        if (!rq->target) return fail(RT_EINVAL, "target is NULL");
        if (rq->problem.spec.nch > kLaunchChannels)
            return fail(RT_EINVAL, "gradient requests take at most %d channels", kLaunchChannels);
        if (rq->grads.d_mlp && !rq->problem.mlp) return fail(RT_EINVAL, "d_mlp requested without a network");
    }
    std::unique_ptr<Req> r(new Req);
    r->rq = *rq;
    const rt_problem &p = rq->problem;
    r->lev_e.assign(p.line.lev_e_k, p.line.lev_e_k + p.line.nlev);
    r->lev_g.assign(p.line.lev_g, p.line.lev_g + p.line.nlev);
    r->vk.assign(p.spec.v_kms, p.spec.v_kms + p.spec.nch);
    r->rq.problem.line.lev_e_k = r->lev_e.data();
    r->rq.problem.line.lev_g = r->lev_g.data();
    r->rq.problem.spec.v_kms = r->vk.data();
    if (p.mlp) {
        r->mlp = *p.mlp;
        r->rq.problem.mlp = &r->mlp;
    }
    // lanes of the request in the persistent launch (kServeSplit per pixel and
    // 16-channel block) against the lanes the launch keeps resident
    const uint64_t device_lanes = (uint64_t)sv->ncu * kServeWorkgroupsPerCU * 256;
    const uint64_t serve_lanes = (uint64_t)p.cam.nx * p.cam.ny * ((p.spec.nch + 15) / 16) * kServeSplit;
    // size of a gradient request in the batched reverse march, counted as two
    // lanes per pixel and 32-channel slice.  Measured per request with the
    // pair form of the march (eight of one shape, batched vs the fused
    // single-request path, ms): 64^2 x 16 x 256 0.41 vs 0.54, 64^2 x 64 x 512
    // 0.59 vs 1.03, 128^2 x 32 x 256 0.52 vs 0.67, but 128^2 x 128 x 384 1.53
    // vs 1.35 and 256^2 x 16 x 256 1.31 vs 1.00: requests under a quarter of
    // the device's resident lanes batch.  The batched march needs its
    // channels uniformly spaced in groups of kGradLaneCB; other requests run
    // on their own stream.
    const uint64_t grad_lanes = (uint64_t)p.cam.nx * p.cam.ny * ((p.spec.nch + kGradSlice - 1) / kGradSlice) * 2;
    double gshift = 0.0;
    if (rq->kind == RT_REQ_FWD_ADJ) {
        r->grad_batch = p.mlp == nullptr && grad_lanes < device_lanes / 4 && grad_batch_grid_fits(p.grid.nr, p.grid.nz) &&
                        group_shift(p.spec.v_kms, p.spec.nch, kGradLanes, kGradLaneCB, &gshift);
        r->own_stream = !r->grad_batch;
    } else {
        r->own_stream = p.mlp != nullptr || serve_lanes >= device_lanes;
    }
    r->footprint = footprint(*rq, r->grad_batch);
    r->ray_samples = (uint64_t)p.cam.nx * p.cam.ny * p.spec.nch * p.nsamp;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(RT_ECANCELED, "server is shutting down");
    if (r->footprint > sv->cfg.hbm_budget_bytes)
        return fail(RT_ETOOBIG, "request needs %llu bytes, budget is %llu", (unsigned long long)r->footprint,
                    (unsigned long long)sv->cfg.hbm_budget_bytes);
    if ((int)sv->pending.size() >= sv->cfg.max_pending) return fail(RT_EAGAIN, "pending queue is full");
    r->id = sv->next_id++;
    r->t_submit = now_ns();
    *ticket = r->id;
    sv->pending.push_back(r.get());
    sv->tickets[r->id] = std::move(r);
    sv->cv.notify_all();
    return RT_OK;
}

static void fill_info(const Req *r, rt_ticket_info *info) {
    info->state = r->state;
    info->status = r->status;
    info->t_submit_ns = r->t_submit;
    info->t_admit_ns = r->t_admit;
    info->t_done_ns = r->t_done;
    info->loss = r->loss;
    info->ray_samples = r->ray_samples;
}

rt_status rt_poll(rt_server *sv, uint64_t ticket, rt_ticket_info *info) {
    if (!sv || !info) return fail(RT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(RT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    fill_info(it->second.get(), info);
    return RT_OK;
}

rt_status rt_wait(rt_server *sv, uint64_t ticket, rt_ticket_info *info, uint64_t timeout_ns) {
    if (!sv || !info) return fail(RT_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(RT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second.get();
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns);
    while (r->state == RT_TICKET_QUEUED || r->state == RT_TICKET_RUNNING) {
        if (sv->cv.wait_until(lk, deadline) == std::cv_status::timeout) break;
    }
    fill_info(r, info);
    return (r->state == RT_TICKET_QUEUED || r->state == RT_TICKET_RUNNING) ? RT_PENDING : RT_OK;
}

rt_status rt_cancel(rt_server *sv, uint64_t ticket) {
    if (!sv) return fail(RT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(RT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second.get();
    if (r->state != RT_TICKET_QUEUED) return fail(RT_EINVAL, "request already admitted or finished");
    for (auto q = sv->pending.begin(); q != sv->pending.end(); ++q)
        if (*q == r) { sv->pending.erase(q); break; }
    r->state = RT_TICKET_CANCELED;
    r->status = RT_ECANCELED;
    r->t_done = now_ns();
    sv->cv.notify_all();
    return RT_OK;
}

rt_status rt_release(rt_server *sv, uint64_t ticket) {
    if (!sv) return fail(RT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(RT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    const int st = it->second->state;
    if (st == RT_TICKET_QUEUED || st == RT_TICKET_RUNNING) return fail(RT_EINVAL, "request has not finished");
    sv->tickets.erase(it);
    return RT_OK;
}

rt_status rt_server_destroy(rt_server *sv) {
    if (!sv) return fail(RT_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        for (Req *r : sv->pending) {
            r->state = RT_TICKET_CANCELED;
            r->status = RT_ECANCELED;
            r->t_done = now_ns();
        }
        sv->pending.clear();
        sv->cv.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    for (Lane &L : sv->lanes) {
        if (L.st) release_stream_workspaces(L.st);
        if (L.st) (void)hipStreamSynchronize(L.st);
        if (L.ev) (void)hipEventDestroy(L.ev);
        if (L.st) (void)hipStreamDestroy(L.st);
        if (L.d_desc) (void)hipFree(L.d_desc);
        if (L.h_desc) (void)hipHostFree(L.h_desc);
        if (L.d_vch) (void)hipFree(L.d_vch);
        if (L.h_vch) (void)hipHostFree(L.h_vch);
        if (L.d_counter) (void)hipFree(L.d_counter);
        if (L.d_loss) (void)hipFree(L.d_loss);
        if (L.h_loss) (void)hipHostFree(L.h_loss);
        if (L.d_gdesc) (void)hipFree(L.d_gdesc);
        if (L.h_gdesc) (void)hipHostFree(L.h_gdesc);
        if (L.d_gcount) (void)hipFree(L.d_gcount);
    }
    delete sv;
    return RT_OK;
}

} // extern "C"
