// Host driver of the batched CG (hisq_cg_batch): many independent problems,
// each with its own lattice, mass, links and tolerance, solved together.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "api_util.hpp"
#include "batch.hpp"

namespace hisq {

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    int fs;
    int nblocks;
    size_t probs, blk, state, mask, partials, flags, scal, fields, total;
    std::vector<size_t> r, p, q, t, ax, t64;
};

BatchLayout batch_layout(int n, const hisq_problem *pr, int inner) {
    BatchLayout L;
    L.fs = inner == HISQ_FP64 ? HISQ_FP64 : HISQ_FP32;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = al256(off + b);
        return o;
    };
    L.nblocks = 0;  // at the smallest block size: the most blocks any choice needs
    for (int j = 0; j < n; ++j) {
        const Geom g = make_geom(pr[j].lat);
        L.nblocks += (g.vh + BATCH_BLOCK_MIN - 1) / BATCH_BLOCK_MIN;
    }
    L.probs = take(sizeof(BatchProb) * n);
    L.blk = take(sizeof(int) * L.nblocks);
    L.state = take(sizeof(CgScalars) * n);
    L.mask = take(sizeof(int) * n);
    L.partials = take(sizeof(double) * L.nblocks);
    L.flags = take(64 * sizeof(unsigned));
    L.scal = take(sizeof(double) * (MAX_BATCH + 8));
    L.fields = off;
    for (int j = 0; j < n; ++j) {
        const Geom g = make_geom(pr[j].lat);
        const size_t fb = field_bytes(g, L.fs, 1), f64 = field_bytes(g, HISQ_FP64, 1);
        L.r.push_back(take(fb));
        L.p.push_back(take(fb));
        L.q.push_back(take(fb));
        L.t.push_back(take(fb));
        L.ax.push_back(take(f64));
        L.t64.push_back(take(f64));
    }
    L.total = off;
    return L;
}

double wall_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum { BF_NACTIVE = 0, BF_NPEND = 1 };

}  // namespace

}  // namespace hisq

using namespace hisq;

extern "C" {

size_t hisq_cg_batch_workspace_bytes(int32_t nproblems, const hisq_problem *problems, hisq_prec inner) {
    if (nproblems < 1 || nproblems > MAX_BATCH || !problems || check_prec(inner) != HISQ_OK ||
        inner == HISQ_FP64R12 || inner == HISQ_FP32R12 || inner == HISQ_FP64W14 || inner == HISQ_FP32W14)
        return 0;
    for (int j = 0; j < nproblems; ++j)
        if (check_lattice(&problems[j].lat) != HISQ_OK)
            return 0;
    return batch_layout(nproblems, problems, inner).total;
}

hisq_status hisq_cg_batch(hisq_context *ctx, int32_t nproblems, const hisq_problem *problems, hisq_prec inner,
                          int32_t max_iter, void *ws, size_t ws_bytes, hisq_solve_info *info, double *latency_s,
                          void *stream) {
    const double t0 = wall_s();
    if (nproblems < 1 || nproblems > MAX_BATCH)
        return fail(HISQ_ERR_INVALID_ARG, "nproblems = %d outside [1, %d]", nproblems, MAX_BATCH);
    hisq_status s = check_ptr(problems, "problems");
    if (s == HISQ_OK) s = check_prec(inner);
    if (s == HISQ_OK &&
        (inner == HISQ_FP64R12 || inner == HISQ_FP32R12 || inner == HISQ_FP64W14 || inner == HISQ_FP32W14))
        s = fail(HISQ_ERR_UNSUPPORTED, "the batched solver takes FP64, FP32 or FP16N links, not compressed ones");
    if (s == HISQ_OK) s = check_ptr(ws, "ws");
    if (s == HISQ_OK && max_iter < 1)
        s = fail(HISQ_ERR_INVALID_ARG, "max_iter = %d must be >= 1", max_iter);
    for (int j = 0; s == HISQ_OK && j < nproblems; ++j) {
        const hisq_problem &P = problems[j];
        s = check_lattice(&P.lat);
        if (s == HISQ_OK && (!std::isfinite(P.mass) || P.mass * P.mass <= 0.0))
            s = fail(HISQ_ERR_INVALID_ARG, "problem %d: mass^2 must be positive", j);
        if (s == HISQ_OK && !(P.tol > 0.0 && P.tol < 1.0))
            s = fail(HISQ_ERR_INVALID_ARG, "problem %d: tol = %g must be in (0, 1)", j, P.tol);
        if (s == HISQ_OK && (!P.links_f64 || !P.b || !P.x || (inner != HISQ_FP64 && !P.links_inner)))
            s = fail(HISQ_ERR_INVALID_ARG, "problem %d: NULL links, b or x", j);
        if (s == HISQ_OK && P.b == P.x)
            s = fail(HISQ_ERR_INVALID_ARG, "problem %d: b and x alias", j);
    }
    if (s == HISQ_OK) s = set_device(ctx);
    if (s != HISQ_OK)
        return s;
    const BatchLayout L = batch_layout(nproblems, problems, inner);
    if (ws_bytes < L.total)
        return fail(HISQ_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, L.total);
    char *W = static_cast<char *>(ws);
    const int n = nproblems;
    const int lp = inner;

    // private stream ordered after the caller's (graphs cannot capture the legacy stream)
    hipStream_t caller = static_cast<hipStream_t>(stream), st = nullptr;
    hipEvent_t ev = nullptr;
    struct Cleanup {
        hipStream_t *st;
        hipEvent_t *ev;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~Cleanup() {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (*st) {
                (void)hipStreamSynchronize(*st);
                (void)hipStreamDestroy(*st);
            }
            if (*ev) (void)hipEventDestroy(*ev);
        }
    } cleanup{&st, &ev};
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
    if (e != hipSuccess)
        return device_fail(e, "stream setup");

    // problem table and work list
    std::vector<BatchProb> probs(n);
    std::vector<int> blk(L.nblocks);
    int nblocks = 0;  // blocks of the chosen work list
    for (int j = 0; j < n; ++j) {
        const hisq_problem &P = problems[j];
        BatchProb &B = probs[j];
        B.g = make_geom(P.lat);
        B.m2 = P.mass * P.mass;
        B.links64 = static_cast<const char *>(P.links_f64);
        B.links_in = inner == HISQ_FP64 ? B.links64 : static_cast<const char *>(P.links_inner);
        B.b = P.b;
        B.x = P.x;
        B.r = W + L.r[j];
        B.p = W + L.p[j];
        B.q = W + L.q[j];
        B.t = W + L.t[j];
        B.ax = W + L.ax[j];
        B.t64 = W + L.t64[j];
    }
    // work list for `bb` sites per block: problem j owns blocks
    // [first_blk, first_blk + nblk); returns the number of blocks.  With
    // `keep`, problems outside it get no blocks (nblk = 0).
    auto assign = [&](int bb, const std::vector<char> *keep = nullptr) -> int {
        int total = 0;
        for (int j = 0; j < n; ++j) {
            const int nb = (keep && !(*keep)[j]) ? 0 : (probs[j].g.vh + bb - 1) / bb;
            probs[j].first_blk = total;
            probs[j].nblk = nb;
            for (int b = 0; b < nb; ++b)
                blk[total + b] = j;
            total += nb;
        }
        return total;
    };
    BatchArgs a{};
    a.probs = reinterpret_cast<const BatchProb *>(W + L.probs);
    a.nprob = n;
    a.blk_prob = reinterpret_cast<const int *>(W + L.blk);
    a.st = reinterpret_cast<CgScalars *>(W + L.state);
    a.mask = reinterpret_cast<int *>(W + L.mask);
    a.partials = reinterpret_cast<double *>(W + L.partials);
    unsigned *flags = reinterpret_cast<unsigned *>(W + L.flags);
    a.nactive = reinterpret_cast<int *>(flags + BF_NACTIVE);
    a.npend = reinterpret_cast<int *>(flags + BF_NPEND);
    a.block = 128;
    double *scal = reinterpret_cast<double *>(W + L.scal);  // [0..n) ||b||^2, [MAX_BATCH] start clock
    int *mask_d = reinterpret_cast<int *>(W + L.mask);

    std::vector<CgScalars> hs(n);
    std::vector<int> mask(n, 1), reliable(n, 0);
    std::vector<double> bnorm2(n), rtrue2(n, 0.0), t_stop(n, 0.0);
    auto push = [&](bool state, bool msk) -> hipError_t {
        hipError_t err = hipSuccess;
        if (state) {
            int nact = 0;
            for (int j = 0; j < n; ++j) nact += hs[j].active != 0;
            err = hipMemcpyAsync(a.st, hs.data(), sizeof(CgScalars) * n, hipMemcpyHostToDevice, st);
            if (err == hipSuccess)
                err = hipMemcpyAsync(flags + BF_NACTIVE, &nact, sizeof nact, hipMemcpyHostToDevice, st);
        }
        if (msk && err == hipSuccess) {
            static const int one = 1;  // a host-driven true-residual pass: let its kernels run
            err = hipMemcpyAsync(mask_d, mask.data(), sizeof(int) * n, hipMemcpyHostToDevice, st);
            if (err == hipSuccess)
                err = hipMemcpyAsync(flags + BF_NPEND, &one, sizeof one, hipMemcpyHostToDevice, st);
        }
        if (err == hipSuccess)
            err = hipStreamSynchronize(st);
        return err;
    };
    auto pull = [&]() -> hipError_t {
        hipError_t err = hipMemcpyAsync(hs.data(), a.st, sizeof(CgScalars) * n, hipMemcpyDeviceToHost, st);
        if (err == hipSuccess)
            err = hipStreamSynchronize(st);
        return err;
    };
    // true residual of the masked problems: r = b - M x (FP64), rho_new = ||r||^2
    auto true_residuals = [&](bool copy_p) -> hipError_t {
        hipError_t err = push(false, true);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_TRUE_DOE, lp, st);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_TRUE_DEO, lp, st);
        if (err == hipSuccess)
            err = launch_batch(a, nblocks, copy_p ? BOP_RESIDUAL_COPY_P : BOP_RESIDUAL, lp, st);
        if (err == hipSuccess) err = pull();
        return err;
    };

    auto upload = [&]() -> hipError_t {
        hipError_t err = hipMemcpyAsync(W + L.probs, probs.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice, st);
        if (err == hipSuccess)
            err = hipMemcpyAsync(W + L.blk, blk.data(), sizeof(int) * nblocks, hipMemcpyHostToDevice, st);
        return err;
    };
    if (e == hipSuccess) e = launch_fill_u32(flags, 64, 0u, st);
    // tile autotuning: time one iteration Dslash of the whole batch at 64, 128
    // and 256 sites per block (vectors zeroed, every problem active) and keep
    // the fastest work list; a larger tile must be 5 % faster to be taken,
    // because the tail of the few long solves, on small lattices, prefers
    // small tiles (uneven batch of 64: 0.921 s at 256, 0.89-0.905 s at 64)
    if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<unsigned *>(W + L.fields), (L.total - L.fields) / 4, 0u, st);
    for (int j = 0; j < n; ++j) {
        CgScalars c{};
        c.active = 1;
        hs[j] = c;
    }
    if (e == hipSuccess) e = push(true, false);
    {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        float best_ms = 1e30f;
        int best = 128;
        for (int bb : {64, 128, 256}) {
            if (e != hipSuccess)
                break;
            a.block = bb;
            nblocks = assign(bb);
            e = upload();
            if (e == hipSuccess) e = launch_batch(a, nblocks, BOP_ITER_DOE, lp, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int k = 0; k < 3 && e == hipSuccess; ++k)
                e = launch_batch(a, nblocks, BOP_ITER_DOE, lp, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms < 0.95f * best_ms) {
                best_ms = ms;
                best = bb;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        a.block = best;
        nblocks = assign(best);
        if (e == hipSuccess) e = upload();
    }
    for (int j = 0; j < n; ++j) {
        CgScalars c{};
        c.active = 0;
        hs[j] = c;
    }
    if (e == hipSuccess) e = push(true, true);
    if (e == hipSuccess) e = launch_batch_bnorm(a, nblocks, scal, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bnorm2.data(), scal, sizeof(double) * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = true_residuals(true);
    if (e != hipSuccess)
        return device_fail(e, "batch setup");
    const double delta = inner == HISQ_FP64 ? 0.0 : RELIABLE_DELTA;
    bool breakdown = false;
    for (int j = 0; j < n; ++j) {
        CgScalars c{};
        rtrue2[j] = hs[j].rho_new;
        c.rtrue2 = rtrue2[j];
        c.rho = rtrue2[j];
        c.rmax2 = rtrue2[j];
        c.target2 = problems[j].tol * problems[j].tol * bnorm2[j];
        c.delta2 = delta * delta;
        c.max_iter = max_iter;
        if (!std::isfinite(bnorm2[j]) || !std::isfinite(rtrue2[j])) {
            c.flag = FLAG_BREAKDOWN;
            breakdown = true;
        } else if (rtrue2[j] <= c.target2) {
            c.flag = FLAG_DONE;
        } else {
            c.flag = FLAG_RUN;
            c.active = 1;
        }
        hs[j] = c;
    }
    e = push(true, false);
    // no problem waits for a true residual yet (the masks of the start are spent)
    std::fill(mask.begin(), mask.end(), 0);
    static const int zero = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(mask_d, mask.data(), sizeof(int) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(flags + BF_NPEND, &zero, sizeof zero, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = launch_batch_clock(scal + MAX_BATCH, st);
    if (e != hipSuccess)
        return device_fail(e, "batch start");

    // graph of one chunk of batched iterations.  Every `check` iterations a
    // true-residual block serves the problems that raised FLAG_CONV or
    // FLAG_RELIABLE since the last one (their mask is set on the device): FP64
    // r = b - A x, then the decision (DONE / MAXIT / residual replacement) and
    // p = r + beta p for the restarted problems, all without the host; the
    // launches of the block do nothing while no problem waits.  A block every
    // 16 iterations (uneven batch of 64: 0.88-0.89 s, against 0.89-0.90 s with
    // the host deciding between chunks); every 4 its idle launches cost more
    // than they save (0.917 s).
    const int chunk = 32, check = 16;
    auto iterate = [&]() -> hipError_t {
        hipError_t err = launch_batch(a, nblocks, BOP_ITER_DOE, lp, st);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_ITER_DEO, lp, st);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_XR, lp, st);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_P, lp, st);
        return err;
    };
    auto tr_block = [&]() -> hipError_t {
        hipError_t err = launch_batch(a, nblocks, BOP_TRUE_DOE, lp, st);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_TRUE_DEO, lp, st);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_RESIDUAL, lp, st);
        if (err == hipSuccess) err = launch_batch(a, nblocks, BOP_RESTART, lp, st);
        return err;
    };
    auto chunk_eager = [&]() -> hipError_t {
        hipError_t err = hipSuccess;
        for (int k = 0; k < chunk && err == hipSuccess; ++k) {
            err = iterate();
            if (err == hipSuccess && (k + 1) % check == 0)
                err = tr_block();
        }
        return err;
    };
    bool use_graph = false;
    auto capture = [&]() {
        if (cleanup.exec) (void)hipGraphExecDestroy(cleanup.exec);
        if (cleanup.graph) (void)hipGraphDestroy(cleanup.graph);
        cleanup.exec = nullptr;
        cleanup.graph = nullptr;
        use_graph = false;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const hipError_t le = chunk_eager();
            hipError_t ce = hipStreamEndCapture(st, &cleanup.graph);
            if (le == hipSuccess && ce == hipSuccess)
                ce = hipGraphInstantiate(&cleanup.exec, cleanup.graph, nullptr, nullptr, 0);
            use_graph = le == hipSuccess && ce == hipSuccess;
        }
        (void)hipGetLastError();
    };
    capture();
    auto terminal = [&](const CgScalars &c) {
        return !c.active && (c.flag == FLAG_DONE || c.flag == FLAG_BREAKDOWN || c.flag == FLAG_MAXIT);
    };
    // Compaction: once the problems still running own at most half of the
    // work list, the list is rebuilt without the finished ones and the chunk
    // graph recaptured, so the tail of a few long solves stops launching
    // blocks for every finished problem (the uneven batch of 64: 0.976 ->
    // 0.932 s).  The stream must be idle (the work list is in use).
    auto compact = [&]() -> hipError_t {
        std::vector<char> keep(n, 0);
        int kept = 0;
        for (int j = 0; j < n; ++j) {
            keep[j] = !terminal(hs[j]);
            if (keep[j])
                kept += (probs[j].g.vh + a.block - 1) / a.block;
        }
        if (kept == 0 || 2 * kept > nblocks)
            return hipSuccess;
        hipError_t err = hipStreamSynchronize(st);
        if (err == hipSuccess) {
            nblocks = assign(a.block, &keep);
            err = upload();
        }
        if (err == hipSuccess)
            err = hipStreamSynchronize(st);
        if (err == hipSuccess)
            capture();
        return err;
    };

    // state read-back into pinned memory, a second chunk queued meanwhile;
    // the pinned buffers are kept for the life of the process and reused by
    // later calls (allocating pinned memory per call took about 0.1 ms)
    struct Pinned {
        CgScalars *p = nullptr;
        size_t bytes = 0;
        hipEvent_t ev[2] = {nullptr, nullptr};
        static std::mutex &mu() {
            static std::mutex m;
            return m;
        }
        static std::vector<std::pair<void *, size_t>> &pool() {
            static std::vector<std::pair<void *, size_t>> v;
            return v;
        }
        hipError_t take(size_t need) {
            std::lock_guard<std::mutex> lk(mu());
            auto &v = pool();
            for (size_t k = 0; k < v.size(); ++k)
                if (v[k].second >= need) {
                    p = static_cast<CgScalars *>(v[k].first);
                    bytes = v[k].second;
                    v.erase(v.begin() + (long)k);
                    return hipSuccess;
                }
            bytes = std::max(need, (size_t)64 << 10);
            void *q = nullptr;
            const hipError_t err = hipHostMalloc(&q, bytes, hipHostMallocDefault);
            p = err == hipSuccess ? static_cast<CgScalars *>(q) : nullptr;
            return err;
        }
        ~Pinned() {
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            if (p) {
                std::lock_guard<std::mutex> lk(mu());
                pool().emplace_back(p, bytes);
            }
        }
    } pin;
    e = pin.take(sizeof(CgScalars) * n * 2);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&pin.ev[k], hipEventDisableTiming);
    if (e != hipSuccess)
        return device_fail(e, "batch read-back setup");
    long launched = 0, read = 0;
    auto launch_chunk = [&]() -> hipError_t {
        hipError_t err = use_graph ? hipGraphLaunch(cleanup.exec, st) : chunk_eager();
        if (err == hipSuccess)
            err = hipMemcpyAsync(pin.p + (launched % 2) * n, a.st, sizeof(CgScalars) * n, hipMemcpyDeviceToHost, st);
        if (err == hipSuccess)
            err = hipEventRecord(pin.ev[launched % 2], st);
        if (err == hipSuccess)
            ++launched;
        return err;
    };
    bool finished = true;
    for (int j = 0; j < n; ++j)
        finished = finished && terminal(hs[j]);
    const long max_chunks = (long)max_iter * check / chunk + 8;
    if (!finished)
        e = launch_chunk();
    while (!finished && e == hipSuccess) {
        if (launched == read + 1 && launched < max_chunks)
            e = launch_chunk();
        if (e == hipSuccess)
            e = hipEventSynchronize(pin.ev[read % 2]);
        if (e != hipSuccess)
            break;
        std::memcpy(hs.data(), pin.p + (read % 2) * n, sizeof(CgScalars) * n);
        ++read;
        finished = true;
        for (int j = 0; j < n; ++j)
            finished = finished && terminal(hs[j]);
        if (finished)
            break;
        if (launched > read) {
            // a chunk is still queued: compact only from an idle stream
            bool want = false;
            int kept = 0;
            for (int j = 0; j < n; ++j)
                if (!terminal(hs[j]))
                    kept += (probs[j].g.vh + a.block - 1) / a.block;
            want = 2 * kept <= nblocks;
            if (want) {
                e = hipEventSynchronize(pin.ev[read % 2]);
                if (e != hipSuccess)
                    break;
                std::memcpy(hs.data(), pin.p + (read % 2) * n, sizeof(CgScalars) * n);
                ++read;
                finished = true;
                for (int j = 0; j < n; ++j)
                    finished = finished && terminal(hs[j]);
                if (finished)
                    break;
                e = compact();
            }
        } else {
            e = compact();
        }
        if (e == hipSuccess && launched == read) {
            if (launched >= max_chunks)
                break;
            e = launch_chunk();
        }
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return device_fail(e, "batch chunk");
    if (launched > read)
        std::memcpy(hs.data(), pin.p + ((launched - 1) % 2) * n, sizeof(CgScalars) * n);
    for (int j = 0; j < n; ++j) {
        if (hs[j].flag == FLAG_DONE) {
            rtrue2[j] = hs[j].rtrue2;
            t_stop[j] = hs[j].spare;
        }
        if (hs[j].flag == FLAG_BREAKDOWN)
            breakdown = true;
        reliable[j] = hs[j].nrel;
    }
    double clock0 = 0.0;
    e = hipMemcpyAsync(&clock0, scal + MAX_BATCH, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int rate_khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx ? ctx->device : 0);
    if (e != hipSuccess)
        return device_fail(e, "batch clock");
    // final true residual of unfinished problems (on the full work list again:
    // compaction may have dropped the ones that stopped at MAXIT or BREAKDOWN)
    bool need = false;
    for (int j = 0; j < n; ++j) {
        mask[j] = hs[j].flag != FLAG_DONE;
        need |= mask[j] != 0;
    }
    if (need) {
        nblocks = assign(a.block);
        e = upload();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return device_fail(e, "batch work list");
        std::vector<CgScalars> before = hs;
        if ((e = true_residuals(false)) != hipSuccess)
            return device_fail(e, "batch final residual");
        for (int j = 0; j < n; ++j) {
            if (mask[j]) {
                rtrue2[j] = hs[j].rho_new;
                before[j].flag = (std::isfinite(rtrue2[j]) && rtrue2[j] <= before[j].target2 &&
                                  before[j].flag != FLAG_BREAKDOWN) ? FLAG_DONE : before[j].flag;
            }
        }
        hs = before;
    }
    hisq_status result = HISQ_OK;
    const double elapsed = wall_s() - t0;
    for (int j = 0; j < n; ++j) {
        if (info) {
            info[j].iterations = hs[j].iters;
            info[j].reliable_updates = reliable[j];
            info[j].true_residual = bnorm2[j] > 0 ? std::sqrt(rtrue2[j] / bnorm2[j]) : std::sqrt(rtrue2[j]);
            info[j].seconds = elapsed;
            info[j].shared_iterations = 0;
            info[j].refine_iterations = 0;
        }
        if (latency_s)
            latency_s[j] = (t_stop[j] > 0.0 && rate_khz > 0) ? (t_stop[j] - clock0) / (rate_khz * 1e3) : 0.0;
        if (hs[j].flag == FLAG_BREAKDOWN)
            result = HISQ_ERR_BREAKDOWN;
        else if (hs[j].flag != FLAG_DONE && result == HISQ_OK)
            result = HISQ_ERR_NOT_CONVERGED;
    }
    if (breakdown)
        result = HISQ_ERR_BREAKDOWN;
    if (result != HISQ_OK)
        fail(result, result == HISQ_ERR_BREAKDOWN ? "batch: a problem broke down" : "batch: not all problems converged");
    return result;
}

}  // extern "C"
