// Host drivers of the conjugate-gradient solvers (paper Sec. 3.2,
// "Inverters"): plain and multi-right-hand-side CG, reliable-update
// mixed-precision CG, and multi-shift CG with per-shift refinement, all for
// the even-site operator M_e = m^2 - D_eo D_oe (+ shift).
//
// CG and reliable-update CG (hisq_cg, the refinement of the multi-shift
// solver) run the single-reduction recurrence of Chronopoulos and Gear, four
// kernels per iteration: D_oe r -> t; w = (m^2 + sigma) r - D_eo t with the
// block partials of Re<r, w>; per column, the sums of those and of the <r, r>
// partials and the scalar step; p = r + beta p, s = w + beta s, x += alpha p,
// r -= alpha s with the <r, r> partials of the new r.  The shared Krylov
// phase of multi-shift CG keeps the two-reduction (Hestenes-Stiefel)
// recurrence, which Jegerlehner's shifted recurrences are written for: five
// kernels, D_oe p; q = A p with the Re<p, q> partials; x, r with the <r, r>
// partials; the one-block scalar update; p = r + beta p.  Chunks of
// iterations are captured once into a HIP graph and replayed; kernels of
// converged right-hand sides do nothing, and the host looks at the device
// state only between chunks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "api_util.hpp"
#include "dslash.hpp"
#include "solver.hpp"

namespace hisq {

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    int fs;  // sloppy field precision (FP64 or FP32)
    int nblk_max;
    size_t state, state2, shifts, ms, flags, scal, partials, dpart, rr, rspart, pspart, r, p, q, w, t, ps, ax, t64,
        t64m, axm, total;
    size_t part_set;  // doubles of one set of <r, r> (or Re <r, s>, <p, s>) partials
};

Layout make_layout(const Geom &g, int inner, int nrhs, int nshift) {
    Layout L;
    L.fs = field_prec_of(inner) == HISQ_FP64 ? HISQ_FP64 : HISQ_FP32;
    L.nblk_max = std::max(g.vh / 4 + 1, blas_blocks(g.vh));  // a Dslash site block holds >= 4 sites
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.state = take(sizeof(CgScalars) * HISQ_MAX_RHS);
    L.state2 = take(sizeof(CgScalars) * HISQ_MAX_RHS);  // second buffer of the fused single-reduction step
    L.shifts = take(sizeof(ShiftScalars) * MAX_SHIFTS);
    L.ms = take(sizeof(MsGlobal));
    L.flags = take(64 * sizeof(unsigned));
    L.scal = take(64 * sizeof(double));
    // the multi-shift refinement solves up to HISQ_MAX_RHS shifts as columns
    const int ncol = std::max(nrhs, std::min(std::max(nshift, 0), (int)HISQ_MAX_RHS));
    L.partials = take(sizeof(double) * (size_t)std::max(ncol, 1) * L.nblk_max);
    // <p, A p> partials (two-reduction CG) or Re <r, A r> partials (single-reduction CG)
    L.dpart = take(sizeof(double) * (size_t)std::max(ncol, 1) * L.nblk_max);
    // single-reduction CG: two sets each of the <r, r>, Re <r, s> and <p, s> partials
    L.part_set = (size_t)std::max(ncol, 1) * cg_vec_blocks(g.vh);
    L.rr = take(sizeof(double) * 2 * L.part_set);
    L.rspart = take(sizeof(double) * 2 * L.part_set);
    L.pspart = take(sizeof(double) * 2 * L.part_set);
    const size_t fb = field_bytes(g, L.fs, 1), fbn = field_bytes(g, L.fs, ncol);
    L.r = take(fbn);
    L.p = take(fbn);
    L.q = take(fbn);  // A p (s of the single-reduction CG)
    L.w = take(fbn);  // A r (single-reduction CG)
    L.t = take(fbn);
    L.ps = take(fb * std::max(nshift, 0));  // one-column fields end to end
    const size_t f64 = field_bytes(g, HISQ_FP64, 1);
    L.ax = take(f64);
    L.t64 = take(f64);
    // several right-hand sides: the true residuals of all columns in one
    // multi-right-hand-side FP64 operator application
    const int nm = nrhs > 1 ? nrhs : 0;
    L.t64m = take(f64 * nm);
    L.axm = take(f64 * nm);
    L.total = off;
    return L;
}

// flags[] slots
// F_NOPEND: no true residual pending; F_TR0 + j: tr_skip of column j;
// F_OFF0 + j: column j inactive (the fused single-reduction step's launch gate)
enum { F_SKIP = 0, F_NOPEND = 2, F_TR0 = 16, F_OFF0 = 32 };
// scal[] slots
enum { S_TMP = 0, S_B = 16, S_R = 32 };  // S_B + j: ||b_j||^2, S_R + j: ||b_j - A x_j||^2

struct Solver {
    hisq_context *ctx = nullptr;
    Geom g{};
    hipStream_t st = nullptr;
    double mass = 0.0;
    const char *links64 = nullptr;
    const char *links_in = nullptr;
    int lp_in = HISQ_FP64;
    Layout L{};
    char *ws = nullptr;
    DslashShape shape64{};
    DslashShape shape64m{};  // FP64 operator on all nrhs columns at once
    DslashShape shape_in{};
    int chunk = 16;
    double iter_us = 100.0;  // estimated time of one iteration

    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    unsigned *flags() const { return at<unsigned>(L.flags); }
    double *scal() const { return at<double>(L.scal); }
    double *partials() const { return at<double>(L.partials); }
    size_t f64_col() const { return field_bytes(g, HISQ_FP64, 1); }
    size_t fs_col() const { return field_bytes(g, L.fs, 1); }

    hisq_status dev(hipError_t e, const char *where) const {
        return e == hipSuccess ? HISQ_OK : device_fail(e, where);
    }

    // out = (m^2 + sigma) in - D_eo D_oe in, FP64, one column; both launches
    // do nothing while skip (nullable) points to a nonzero value.
    hipError_t m64(double sigma, const void *in, void *out, const int *skip) {
        DslashParams prm{};
        prm.g = g;
        prm.nrhs = 1;
        prm.links = links64;
        prm.skip = skip;
        prm.out_parity = 1;
        prm.in = in;
        prm.out = at<void>(L.t64);
        hipError_t e = launch_dslash(prm, HISQ_FP64, HISQ_FP64, EPI_PLAIN, shape64, st);
        if (e != hipSuccess)
            return e;
        prm.out_parity = 0;
        prm.in = at<void>(L.t64);
        prm.out = out;
        prm.y = in;
        prm.ad = -1.0;
        prm.ay = mass * mass + sigma;
        return launch_dslash(prm, HISQ_FP64, HISQ_FP64, EPI_AXPY, shape64, st);
    }
    hisq_status apply_m64(double sigma, const void *in, void *out) { return dev(m64(sigma, in, out, nullptr), "M_e"); }

    hisq_status read_double(const double *d, double *h) {
        hipError_t e = hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        return dev(e, "read scalar");
    }

    // ||v||^2 of an FP64 column.
    hisq_status norm2(const void *v, double *out) {
        hisq_status s = dev(launch_norm2(g.vh, v, partials(), scal() + S_TMP, st), "norm2");
        return s == HISQ_OK ? read_double(scal() + S_TMP, out) : s;
    }

    // r_sloppy[col] = b - (M + sigma) x and its FP64 norm^2.
    hisq_status true_residual(double sigma, const void *b, const void *x, void *r_sloppy, double *out2) {
        hisq_status s = apply_m64(sigma, x, at<void>(L.ax));
        if (s != HISQ_OK)
            return s;
        s = dev(launch_residual(g.vh, L.fs, b, at<void>(L.ax), r_sloppy, partials(), scal() + S_TMP, st),
                "residual");
        return s == HISQ_OK ? read_double(scal() + S_TMP, out2) : s;
    }

    // One single-reduction CG iteration for nrhs columns (column j solving
    // (M_e + sigma[j]) x = b): D_oe r; w = A r with the Re <r, w> partials;
    // the per-column scalar step and the vector update, as two launches, or
    // as one (fused: every block sums its column's partials; the state
    // alternates between the two buffers, iteration k reading buffer k % 2,
    // and the Dslash launches are gated per column).
    hipError_t iteration_sr(const CgVecParams &vp, const double *sigma, int nrhs, int after_check, bool fused,
                            int k) {
        DslashParams prm{};
        prm.g = g;
        prm.nrhs = nrhs;
        prm.links = links_in;
        int *off = reinterpret_cast<int *>(flags() + F_OFF0);
        if (fused)
            prm.col_skip = off;
        else
            prm.skip = reinterpret_cast<const int *>(flags() + F_SKIP);
        prm.out_parity = 1;
        prm.in = vp.r;
        prm.out = at<void>(L.t);
        hipError_t e = launch_dslash(prm, lp_in, L.fs, EPI_PLAIN, shape_in, st);
        if (e != hipSuccess)
            return e;
        prm.out_parity = 0;
        prm.in = at<void>(L.t);
        prm.out = const_cast<void *>(vp.w);
        prm.y = vp.r;
        prm.ad = -1.0;
        prm.ay = mass * mass + sigma[0];
        prm.ay_per_rhs = 1;
        for (int j = 0; j < nrhs; ++j)
            prm.ay_rhs[j] = mass * mass + sigma[j];
        prm.partials = const_cast<double *>(vp.rw_part);
        prm.dot_out = nullptr;  // summed by the scalar step
        e = launch_dslash(prm, lp_in, L.fs, EPI_AXPY_DOT, shape_in, st);
        if (e != hipSuccess)
            return e;
        if (!fused)
            return launch_cgcg_step(vp, L.fs, after_check, st);
        CgScalars *b0 = at<CgScalars>(L.state), *b1 = at<CgScalars>(L.state2);
        return launch_cgcg_fused(vp, L.fs, k & 1 ? b1 : b0, k & 1 ? b0 : b1, off, after_check, k & 1, st);
    }

    // The five kernels of one two-reduction iteration for nrhs right-hand
    // sides, column j solving (M_e + sigma[j]) x = b.
    hipError_t iteration(const CgVecParams &vp, const double *sigma, int nrhs) {
        DslashParams prm{};
        prm.g = g;
        prm.nrhs = nrhs;
        prm.links = links_in;
        prm.skip = reinterpret_cast<const int *>(flags() + F_SKIP);
        prm.out_parity = 1;
        prm.in = vp.p;
        prm.out = at<void>(L.t);
        hipError_t e = launch_dslash(prm, lp_in, L.fs, EPI_PLAIN, shape_in, st);
        if (e != hipSuccess)
            return e;
        prm.out_parity = 0;
        prm.in = at<void>(L.t);
        prm.out = const_cast<void *>(vp.q);
        prm.y = vp.p;
        prm.ad = -1.0;
        prm.ay = mass * mass + sigma[0];
        prm.ay_per_rhs = 1;
        for (int j = 0; j < nrhs; ++j)
            prm.ay_rhs[j] = mass * mass + sigma[j];
        // the <p, A p> partials are summed inside the x/r update and the
        // finalize kernel (no reduction launch of their own)
        prm.partials = at<double>(L.dpart);
        prm.dot_out = nullptr;
        e = launch_dslash(prm, lp_in, L.fs, EPI_AXPY_DOT, shape_in, st);
        if (e != hipSuccess)
            return e;
        CgVecParams v2 = vp;
        v2.pq_part = at<double>(L.dpart);
        v2.pq_nblk = dslash_partial_blocks(g, shape_in);
        e = launch_cg_xr(v2, L.fs, st);
        if (e != hipSuccess)
            return e;
        return launch_cg_p(vp, L.fs, 0, nrhs, st);
    }
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// A private non-blocking stream ordered after the caller's stream (graphs
// cannot be captured on the legacy default stream).  Each thread keeps one
// such stream and event per device for the life of the process (a solve
// synchronizes its stream before it returns, so the next solve of the thread
// finds it idle); creating and destroying them per solve cost about 0.1 ms.
struct StreamGuard {
    hipStream_t caller = nullptr, own = nullptr;
    hipEvent_t ev = nullptr;
    hipError_t init(hipStream_t c) {
        caller = c;
        struct Slot {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
        };
        static thread_local std::vector<Slot> *slots = new std::vector<Slot>();
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess)
            return e;
        if ((int)slots->size() <= dev)
            slots->resize(dev + 1);
        Slot &sl = (*slots)[dev];
        if (!sl.st) {
            e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
            if (e != hipSuccess) {
                sl.st = nullptr;
                return e;
            }
        }
        if (!sl.ev) {
            e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                sl.ev = nullptr;
                return e;
            }
        }
        own = sl.st;
        ev = sl.ev;
        e = hipEventRecord(ev, caller);
        if (e != hipSuccess)
            return e;
        return hipStreamWaitEvent(own, ev, 0);
    }
    ~StreamGuard() {
        if (own)
            (void)hipStreamSynchronize(own);
    }
};

// Instantiated chunk graphs of earlier solves on this thread, reused when a
// solve repeats every value its launches were captured with (lattice, mass,
// shifts, links, fields, workspace layout, launch shapes, chunk length): the
// kernels read the Krylov state and their flags from device memory, so a
// chunk graph is a function of those values alone.  Eight entries, the least
// recently used evicted; a solve synchronizes its stream before it returns,
// so no evicted graph is still running.  Capturing and instantiating a chunk
// cost 0.1-0.2 ms per solve.
class ChunkGraphCache {
  public:
    static ChunkGraphCache &mine() {
        static thread_local ChunkGraphCache *c = new ChunkGraphCache();
        return *c;
    }
    hipGraphExec_t find(const std::vector<uint64_t> &key) {
        for (Entry &en : e_)
            if (en.key == key) {
                en.used = ++tick_;
                return en.exec;
            }
        return nullptr;
    }
    void put(const std::vector<uint64_t> &key, hipGraphExec_t exec) {
        if (e_.size() >= kMax) {
            size_t lru = 0;
            for (size_t k = 1; k < e_.size(); ++k)
                if (e_[k].used < e_[lru].used)
                    lru = k;
            (void)hipGraphExecDestroy(e_[lru].exec);
            e_.erase(e_.begin() + (long)lru);
        }
        e_.push_back(Entry{key, exec, ++tick_});
    }

  private:
    static constexpr size_t kMax = 8;
    struct Entry {
        std::vector<uint64_t> key;
        hipGraphExec_t exec;
        uint64_t used;
    };
    std::vector<Entry> e_;
    uint64_t tick_ = 0;
};

struct GraphChunk {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    ~GraphChunk() {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
    }
};

}  // namespace

size_t cg_workspace_bytes(const Geom &g, int inner, int nrhs, int nshift) {
    return make_layout(g, inner, nrhs, nshift).total;
}

// The right-hand sides of one CG run: column j solves (M_e + sigma[j]) x[j] =
// b[j] to tol[j] (packed FP64 fields; x holds the initial guess on entry).
struct Columns {
    const void *b[HISQ_MAX_RHS];
    void *x[HISQ_MAX_RHS];
    double sigma[HISQ_MAX_RHS];
    double tol[HISQ_MAX_RHS];
};

// Pinned host slots for reading the solver state back without stalling the
// stream; kept for the life of the process and reused by later solves.
class PinnedSlots {
  public:
    static constexpr int N = 2;
    PinnedSlots() {
        std::lock_guard<std::mutex> lk(mu());
        if (!pool().empty()) {
            buf_ = pool().back();
            pool().pop_back();
        } else if (hipHostMalloc(reinterpret_cast<void **>(&buf_), sizeof(CgScalars) * HISQ_MAX_RHS * N,
                                 hipHostMallocDefault) != hipSuccess) {
            buf_ = nullptr;
        }
    }
    ~PinnedSlots() {
        if (buf_) {
            std::lock_guard<std::mutex> lk(mu());
            pool().push_back(buf_);
        }
    }
    bool ok() const { return buf_ != nullptr; }
    CgScalars *slot(int k) const { return buf_ + (size_t)(k % N) * HISQ_MAX_RHS; }

  private:
    CgScalars *buf_ = nullptr;
    static std::mutex &mu() {
        static std::mutex m;
        return m;
    }
    static std::vector<CgScalars *> &pool() {
        static std::vector<CgScalars *> p;
        return p;
    }
};

bool terminal(const CgScalars &c) {
    return !c.active && (c.flag == FLAG_DONE || c.flag == FLAG_BREAKDOWN || c.flag == FLAG_MAXIT);
}

// Single-reduction CG / reliable-update CG for nrhs columns.  info[nrhs] is
// filled.
//
// The device runs the whole recurrence: every `check` iterations a
// true-residual block forms r_j = b_j - A x_j in FP64 (with the partials of
// its norm in the column's <r, r> slots) for each column that raised
// FLAG_CONV or FLAG_RELIABLE since the last block (the kernels of the other
// columns do nothing), and the scalar step of the next iteration decides DONE
// / MAXIT / residual replacement, so a reliable update needs no host round
// trip.
// Chunks of iterations (a multiple of `check`, each ending with a block) are
// replayed from one HIP graph; the host keeps a second chunk queued while it
// reads the state of the previous one, and stops when every column is done.
static hisq_status run_cg(Solver &S, const Columns &C, int nrhs, int max_iter, double delta,
                          hisq_solve_info *info, const int *prior_iters) {
    const double t0 = now_s();
    const Geom &g = S.g;
    const Layout &L = S.L;
    hipStream_t st = S.st;
    CgScalars *dst = S.at<CgScalars>(L.state);
    std::vector<CgScalars> hs(nrhs);
    std::vector<double> bnorm2(nrhs), rtrue2(nrhs);
    hisq_status s = S.dev(launch_fill_u32(S.flags(), 64, 0u, st), "fill");
    if (s != HISQ_OK)
        return s;

    char *rs = S.at<char>(L.r);
    S.shape_in = pick_shape(S.ctx, g, S.lp_in, L.fs, nrhs);
    const int nb = cg_vec_blocks(g.vh);  // <r, r> partials per column
    double *rr = S.at<double>(L.rr);
    bool breakdown = false;
    // ||b_j||^2, and r_j = b_j - A x_j with its <r, r> partials where the
    // first scalar step reads them and its FP64 norm, for every column; one
    // read-back of the norms for the decisions below
    for (int j = 0; j < nrhs; ++j) {
        hipError_t e = launch_norm2(g.vh, C.b[j], S.partials(), S.scal() + S_B + j, st);
        if (e == hipSuccess)
            e = S.m64(C.sigma[j], C.x[j], S.at<void>(L.ax), nullptr);
        if (e == hipSuccess)
            e = launch_residual_cols(g.vh, 1, nrhs, j, L.fs, C.b[j], S.at<void>(L.ax), rs, rr + (size_t)j * nb,
                                     nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, st);
        if (e == hipSuccess)
            e = launch_sum_partials(rr + (size_t)j * nb, 1, nb, S.scal() + S_R + j, 1, nullptr, st);
        if ((s = S.dev(e, "initial residual")) != HISQ_OK)
            return s;
    }
    {
        double norms[S_R + HISQ_MAX_RHS - S_B];
        hipError_t e = hipMemcpyAsync(norms, S.scal() + S_B, sizeof(norms), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if ((s = S.dev(e, "initial residual norms")) != HISQ_OK)
            return s;
        for (int j = 0; j < nrhs; ++j) {
            bnorm2[j] = norms[j];
            rtrue2[j] = norms[S_R - S_B + j];
        }
    }
    for (int j = 0; j < nrhs; ++j) {
        CgScalars c{};
        c.rho = rtrue2[j];
        c.rmax2 = rtrue2[j];
        c.rtrue2 = rtrue2[j];
        c.target2 = C.tol[j] * C.tol[j] * bnorm2[j];
        c.delta2 = delta * delta;
        c.max_iter = max_iter;
        c.iters = 0;
        c.restart = 1;  // the first step starts the directions: p = r, s = A r
        const bool bad = !std::isfinite(bnorm2[j]) || !std::isfinite(rtrue2[j]);
        if (bad) {
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
    int *trf = reinterpret_cast<int *>(S.flags() + F_TR0);
    {
        int any = 0;
        for (int j = 0; j < nrhs; ++j)
            any |= hs[j].active;
        std::vector<unsigned> fl(F_OFF0 + HISQ_MAX_RHS, 1u);
        fl[F_SKIP] = any ? 0u : 1u;
        for (int j = 0; j < nrhs; ++j)
            fl[F_OFF0 + j] = hs[j].active ? 0u : 1u;
        hipError_t e = hipMemcpyAsync(dst, hs.data(), sizeof(CgScalars) * nrhs, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.flags(), fl.data(), sizeof(unsigned) * fl.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if ((s = S.dev(e, "push state")) != HISQ_OK)
            return s;
    }

    CgVecParams vp{};
    vp.vh = g.vh;
    vp.nrhs = nrhs;
    for (int j = 0; j < nrhs; ++j)
        vp.x[j] = C.x[j];
    vp.r = rs;
    vp.p = S.at<void>(L.p);
    vp.s = S.at<void>(L.q);
    vp.w = S.at<void>(L.w);
    vp.st = dst;
    vp.partials = S.partials();
    vp.rr_part = rr;
    vp.rs_part = S.at<double>(L.rspart);
    vp.ps_part = S.at<double>(L.pspart);
    vp.rr_nblk = nb;
    vp.rw_part = S.at<double>(L.dpart);
    vp.rw_nblk = dslash_partial_blocks(g, S.shape_in);
    // one launch for the scalar and vector steps when every block can afford
    // to sum its column's partials itself (measured: 32^3x8 and smaller);
    // FP32 fields of several columns take the two-launch step, whose vector
    // kernel reads them in column pairs
    const bool fused = vp.rw_nblk <= 2048 && nb <= 2048 && !(L.fs == HISQ_FP32 && nrhs >= 2);
    vp.part_buf = fused ? L.part_set : 0;
    int *col_off = reinterpret_cast<int *>(S.flags() + F_OFF0);
    vp.skip = reinterpret_cast<int *>(S.flags() + F_SKIP);
    vp.tr_skip = trf;
    int *nopend = reinterpret_cast<int *>(S.flags() + F_NOPEND);
    vp.nopend = nopend;
    vp.nshift = 0;

    // true-residual block: columns that wait for one get r = b - A x and the
    // FP64 partials of ||r||^2 in their <r, r> slots (column j's at
    // rr + j * nb), which the next scalar step reads.  When the columns of x
    // and b are one packed multi-column field each (hisq_cg), A x is formed
    // for all of them by one multi-right-hand-side FP64 operator application
    // whenever any column waits (the links are read once, not once per
    // column); otherwise column by column.
    const size_t c64 = S.f64_col();
    bool packed = nrhs > 1;
    for (int j = 1; j < nrhs && packed; ++j)
        packed = static_cast<const char *>(C.x[j]) == static_cast<const char *>(C.x[0]) + j * c64 &&
                 static_cast<const char *>(C.b[j]) == static_cast<const char *>(C.b[0]) + j * c64;
    auto tr_block = [&]() -> hipError_t {
        if (packed) {
            DslashParams prm{};
            prm.g = g;
            prm.nrhs = nrhs;
            prm.links = S.links64;
            if (fused)
                prm.col_skip = trf;
            else
                prm.skip = nopend;
            prm.out_parity = 1;
            prm.in = C.x[0];
            prm.out = S.at<void>(L.t64m);
            hipError_t e = launch_dslash(prm, HISQ_FP64, HISQ_FP64, EPI_PLAIN, S.shape64m, st);
            if (e != hipSuccess)
                return e;
            prm.out_parity = 0;
            prm.in = S.at<void>(L.t64m);
            prm.out = S.at<void>(L.axm);
            prm.y = C.x[0];
            prm.ad = -1.0;
            prm.ay = S.mass * S.mass + C.sigma[0];
            prm.ay_per_rhs = 1;
            for (int j = 0; j < nrhs; ++j)
                prm.ay_rhs[j] = S.mass * S.mass + C.sigma[j];
            e = launch_dslash(prm, HISQ_FP64, HISQ_FP64, EPI_AXPY, S.shape64m, st);
            if (e == hipSuccess)
                e = launch_residual_cols(g.vh, nrhs, nrhs, 0, L.fs, C.b[0], S.at<void>(L.axm), rs, rr, trf, vp.s, vp.p,
                                         vp.rs_part, vp.ps_part, fused ? nullptr : vp.skip,
                                         fused ? col_off : nullptr, st);
            return e;
        }
        for (int j = 0; j < nrhs; ++j) {
            hipError_t e = S.m64(C.sigma[j], C.x[j], S.at<void>(L.ax), trf + j);
            if (e == hipSuccess)
                e = launch_residual_cols(g.vh, 1, nrhs, j, L.fs, C.b[j], S.at<void>(L.ax), rs,
                                         rr + (size_t)j * nb, trf + j, vp.s, vp.p, vp.rs_part + (size_t)j * nb,
                                         vp.ps_part + (size_t)j * nb, fused ? nullptr : vp.skip,
                                         fused ? col_off + j : nullptr, st);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    };
    // iterations between blocks: a flagged column idles until the next one.
    // Chunks of about 0.5 ms (measured: longer chunks overshoot more at the
    // end of a solve).  FP64 iterations flag only at convergence, so they need
    // one block per chunk.  Near the end of a solve (the residual trend
    // predicts fewer iterations than a chunk) short tail chunks of `unit`
    // iterations and one block follow instead, so the iterations launched
    // after convergence are at most those of two tails.
    const int unit = delta > 0.0 ? 4 : 8;
    const int chunk = unit * std::max(1, (int)std::lround(500.0 / (unit * S.iter_us)));
    const int check = delta > 0.0 ? 4 : chunk;
    // a chunk ends with a check block, so the first scalar step of every
    // chunk, and the one after each block, decides the waiting columns; every
    // chunk has an even number of iterations, so each one starts from state
    // buffer 0 and partial set 0 of the fused step
    auto run_iters = [&](int n, int chk) -> hipError_t {
        hipError_t e = hipSuccess;
        for (int k = 0; k < n && e == hipSuccess; ++k) {
            e = S.iteration_sr(vp, C.sigma, nrhs, k % chk == 0 ? 1 : 0, fused, k);
            if (e == hipSuccess && (k + 1) % chk == 0)
                e = tr_block();
        }
        return e;
    };

    bool any_active = false;
    for (int j = 0; j < nrhs; ++j)
        any_active |= hs[j].active != 0;
    // the graphs of the chunk and of the tail, from this thread's cache when a
    // solve with the same launch values ran before
    std::vector<uint64_t> key;
    {
        auto add = [&](uint64_t v) { key.push_back(v); };
        auto addp = [&](const void *q) { add((uint64_t)(uintptr_t)q); };
        auto addd = [&](double d) {
            uint64_t u;
            std::memcpy(&u, &d, sizeof u);
            add(u);
        };
        int dev = 0;
        (void)hipGetDevice(&dev);
        for (int v : {dev, g.nx, g.ny, g.nz, g.nt, g.t_bc, nrhs, S.lp_in, L.fs, chunk, check, unit, fused ? 1 : 0,
                      packed ? 1 : 0, L.nblk_max})
            add((uint64_t)(int64_t)v);
        addd(S.mass);
        for (int j = 0; j < nrhs; ++j) {
            addd(C.sigma[j]);
            addp(C.b[j]);
            addp(C.x[j]);
        }
        addp(S.links64);
        addp(S.links_in);
        addp(S.ws);
        for (size_t o : {L.state, L.state2, L.shifts, L.ms, L.flags, L.scal, L.partials, L.dpart, L.rr, L.rspart,
                         L.pspart, L.r, L.p, L.q, L.w, L.t, L.ps, L.ax, L.t64, L.t64m, L.axm, L.total, L.part_set})
            add(o);
        for (const DslashShape &sh : {S.shape_in, S.shape64, S.shape64m})
            for (int v : {sh.variant, sh.nin, sh.block, sh.xcd_remap})
                add((uint64_t)(int64_t)v);
    }
    hipGraphExec_t exec_chunk = nullptr, exec_tail = nullptr;
    auto graph_of = [&](int n, int chk, int tag) -> hipGraphExec_t {
        std::vector<uint64_t> k = key;
        k.push_back((uint64_t)tag);
        ChunkGraphCache &cache = ChunkGraphCache::mine();
        if (hipGraphExec_t x = cache.find(k))
            return x;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t le = run_iters(n, chk);
            e = hipStreamEndCapture(st, &graph);
            if (le == hipSuccess && e == hipSuccess)
                e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (le != hipSuccess || e != hipSuccess)
                exec = nullptr;
        }
        if (graph)
            (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        if (exec)
            cache.put(k, exec);
        return exec;
    };
    if (any_active) {
        exec_chunk = graph_of(chunk, check, 0);
        exec_tail = graph_of(unit, unit, 1);
    }

    PinnedSlots pin;
    if (any_active && !pin.ok())
        return fail(HISQ_ERR_DEVICE, "hipHostMalloc of the state read-back slots failed");
    hipEvent_t ev[PinnedSlots::N] = {};
    struct EventsGuard {
        hipEvent_t *e;
        ~EventsGuard() {
            for (int k = 0; k < PinnedSlots::N; ++k)
                if (e[k])
                    (void)hipEventDestroy(e[k]);
        }
    } evg{ev};
    for (int k = 0; any_active && k < PinnedSlots::N; ++k)
        if ((s = S.dev(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming), "event")) != HISQ_OK)
            return s;

    long launched = 0, read = 0, launched_iters = 0;
    auto launch_chunk = [&](bool tail) -> hipError_t {
        const int n = tail ? unit : chunk;
        hipGraphExec_t x = tail ? exec_tail : exec_chunk;
        hipError_t e = x ? hipGraphLaunch(x, st) : run_iters(n, tail ? unit : check);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pin.slot((int)launched), dst, sizeof(CgScalars) * nrhs, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipEventRecord(ev[launched % PinnedSlots::N], st);
        if (e == hipSuccess) {
            ++launched;
            launched_iters += n;
        }
        return e;
    };
    // every real iteration advances some column's count, and a column that
    // keeps failing its true-residual check still advances once per block
    // (at least one per `check` iterations, chunks and tails alike)
    const long max_launch_iters = (long)max_iter * check + 4L * chunk;
    std::vector<double> prev_rho(nrhs, 0.0);
    std::vector<int> prev_it(nrhs, 0);
    bool near_end = false;
    hipError_t e = hipSuccess;
    if (any_active)
        e = launch_chunk(false);
    bool finished = !any_active;
    while (!finished && e == hipSuccess) {
        // queue the next chunk (a tail near the end) while this one runs
        if (launched == read + 1 && launched_iters < max_launch_iters)
            e = launch_chunk(near_end);
        if (e == hipSuccess)
            e = hipEventSynchronize(ev[read % PinnedSlots::N]);
        if (e != hipSuccess)
            break;
        std::memcpy(hs.data(), pin.slot((int)read), sizeof(CgScalars) * nrhs);
        ++read;
        finished = true;
        double worst = 0.0;  // most iterations any column still needs (estimate)
        for (int j = 0; j < nrhs; ++j) {
            const CgScalars &c = hs[j];
            if (terminal(c))
                continue;
            finished = false;
            const int dit = c.iters - prev_it[j];
            if (dit > 0 && prev_rho[j] > c.rho && c.rho > 0.0 && c.target2 > 0.0) {
                const double rate = std::log(prev_rho[j] / c.rho) / dit;
                worst = std::max(worst, std::log(c.rho / c.target2) / rate);
            } else {
                worst = 1e30;
            }
            prev_rho[j] = c.rho;
            prev_it[j] = c.iters;
        }
        // the queued chunk still runs: near the end if fewer than two chunks remain
        near_end = worst < 2.0 * chunk;
        if (!finished && launched == read) {
            if (launched_iters >= max_launch_iters)
                break;
            e = launch_chunk(near_end);
        }
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return device_fail(e, "cg chunk");
    if (launched > read)
        std::memcpy(hs.data(), pin.slot((int)(launched - 1)), sizeof(CgScalars) * nrhs);

    // final report
    hisq_status result = HISQ_OK;
    for (int j = 0; j < nrhs; ++j) {
        CgScalars &c = hs[j];
        if (c.flag == FLAG_DONE) {
            rtrue2[j] = c.rtrue2;
        } else {
            double r2 = 0.0;
            // (the sloppy r is not needed any more: scratch for the residual)
            if ((s = S.true_residual(C.sigma[j], C.b[j], C.x[j], rs, &r2)) != HISQ_OK)
                return s;
            rtrue2[j] = r2;
            if (std::isfinite(r2) && r2 <= c.target2 && c.flag != FLAG_BREAKDOWN)
                c.flag = FLAG_DONE;
        }
        if (info) {
            info[j].iterations = c.iters + (prior_iters ? prior_iters[j] : 0);
            info[j].reliable_updates = c.nrel;
            info[j].true_residual = bnorm2[j] > 0 ? std::sqrt(rtrue2[j] / bnorm2[j]) : std::sqrt(rtrue2[j]);
            info[j].seconds = now_s() - t0;
            // a refinement after a multi-shift Krylov phase reports both parts
            info[j].shared_iterations = prior_iters ? prior_iters[j] : 0;
            info[j].refine_iterations = prior_iters ? c.iters : 0;
        }
        if (c.flag == FLAG_BREAKDOWN)
            breakdown = true;
        else if (c.flag != FLAG_DONE && result == HISQ_OK)
            result = HISQ_ERR_NOT_CONVERGED;
    }
    if (breakdown)
        result = HISQ_ERR_BREAKDOWN;
    if (result == HISQ_ERR_NOT_CONVERGED)
        fail(result, "true residual above tolerance after %d iterations", max_iter);
    if (result == HISQ_ERR_BREAKDOWN)
        fail(result, "CG breakdown: <p, A p> not positive or non-finite values");
    return result;
}

// Multi-shift CG (Sec. 3.2: one Krylov space built on the smallest shift,
// the other shifts advanced by Jegerlehner's zeta recurrences in FP64), then
// per-shift refinement by (reliable-update) CG from x_k where the FP64 true
// residual is still above tol_k.  Without `refine` the call ends after the
// shared Krylov phase and reports each x_k's FP64 true residual.
static hisq_status run_multishift(Solver &S, int nshift, const double *shifts, const void *b, void *const *x,
                                  const double *tol, int max_iter, double delta, hisq_solve_info *info,
                                  bool refine) {
    const double t0 = now_s();
    const Geom &g = S.g;
    const Layout &L = S.L;
    hipStream_t st = S.st;
    hisq_status s;
    int base = 0;
    for (int k = 1; k < nshift; ++k)
        if (shifts[k] < shifts[base])
            base = k;
    std::vector<int> others;
    for (int k = 0; k < nshift; ++k)
        if (k != base)
            others.push_back(k);
    const int no = (int)others.size();

    if ((s = S.dev(launch_fill_u32(S.flags(), 64, 0u, st), "fill")) != HISQ_OK)
        return s;
    double bnorm2 = 0.0;
    if ((s = S.norm2(b, &bnorm2)) != HISQ_OK)
        return s;
    const size_t c64 = S.f64_col();
    for (int k = 0; k < nshift; ++k)
        if ((s = S.dev(launch_fill_u32(static_cast<unsigned *>(x[k]), c64 / 4, 0u, st), "zero x")) != HISQ_OK)
            return s;
    std::vector<int> krylov_iters(nshift, 0);
    if (!std::isfinite(bnorm2)) {
        for (int k = 0; k < nshift; ++k)
            if (info) info[k] = hisq_solve_info{0, 0, NAN, now_s() - t0, 0, 0};
        return fail(HISQ_ERR_BREAKDOWN, "non-finite source");
    }
    if (bnorm2 > 0.0) {
        void *rs = S.at<void>(L.r);
        if ((s = S.dev(launch_copy(g.vh, 1, HISQ_FP64, L.fs, b, rs, st), "copy")) != HISQ_OK)
            return s;
        if ((s = S.dev(launch_copy(g.vh, 1, L.fs, L.fs, rs, S.at<void>(L.p), st), "copy")) != HISQ_OK)
            return s;
        for (int j = 0; j < no; ++j)
            if ((s = S.dev(launch_copy(g.vh, 1, L.fs, L.fs, rs, S.at<char>(L.ps) + j * S.fs_col(), st), "copy")) !=
                HISQ_OK)
                return s;
        CgScalars c{};
        c.rho = bnorm2;
        c.rmax2 = bnorm2;
        c.target2 = tol[base] * tol[base] * bnorm2;
        c.delta2 = 0.0;
        c.max_iter = max_iter;
        c.active = 1;
        c.flag = FLAG_RUN;
        std::vector<ShiftScalars> sh(std::max(no, 1));
        for (int j = 0; j < no; ++j) {
            ShiftScalars z{};
            z.s = shifts[others[j]] - shifts[base];
            z.zeta = z.zeta_old = z.zeta_new = 1.0;
            z.target2 = tol[others[j]] * tol[others[j]] * bnorm2;
            z.active = 1;
            sh[j] = z;
        }
        MsGlobal ms{1.0, 0.0, no, 0};
        CgScalars *dst = S.at<CgScalars>(L.state);
        ShiftScalars *dsh = S.at<ShiftScalars>(L.shifts);
        MsGlobal *dms = S.at<MsGlobal>(L.ms);
        hipError_t e = hipMemcpyAsync(dst, &c, sizeof c, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && no > 0)
            e = hipMemcpyAsync(dsh, sh.data(), sizeof(ShiftScalars) * no, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dms, &ms, sizeof ms, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return device_fail(e, "multishift setup");

        CgVecParams vp{};
        vp.vh = g.vh;
        vp.nrhs = 1;
        vp.x[0] = x[base];
        vp.r = rs;
        vp.p = S.at<void>(L.p);
        vp.q = S.at<void>(L.q);
        vp.st = dst;
        vp.partials = S.partials();
        vp.skip = reinterpret_cast<int *>(S.flags() + F_SKIP);
        vp.tr_skip = reinterpret_cast<int *>(S.flags() + F_TR0);  // written, not read, here
        vp.nshift = no;
        vp.sh = dsh;
        vp.ms = dms;
        for (int j = 0; j < no; ++j)
            vp.xs[j] = x[others[j]];
        vp.ps = S.at<void>(L.ps);

        GraphChunk gc;
        bool use_graph = false;
        {
            hipError_t ce = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (ce == hipSuccess) {
                hipError_t le = hipSuccess;
                for (int k = 0; k < S.chunk && le == hipSuccess; ++k)
                    le = S.iteration(vp, &shifts[base], 1);
                ce = hipStreamEndCapture(st, &gc.graph);
                if (le == hipSuccess && ce == hipSuccess)
                    ce = hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0);
                use_graph = le == hipSuccess && ce == hipSuccess;
            }
            (void)hipGetLastError();
        }
        for (int chunk = 0; chunk < max_iter + 64 && c.active; ++chunk) {
            e = use_graph ? hipGraphLaunch(gc.exec, st) : hipSuccess;
            for (int k = 0; !use_graph && k < S.chunk && e == hipSuccess; ++k)
                e = S.iteration(vp, &shifts[base], 1);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&c, dst, sizeof c, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipStreamSynchronize(st);
            if (e != hipSuccess)
                return device_fail(e, "multishift chunk");
        }
        if (no > 0) {
            e = hipMemcpyAsync(sh.data(), dsh, sizeof(ShiftScalars) * no, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipStreamSynchronize(st);
            if (e != hipSuccess)
                return device_fail(e, "multishift state");
        }
        krylov_iters[base] = c.iters;
        for (int j = 0; j < no; ++j)
            krylov_iters[others[j]] = sh[j].iters;
        if (c.flag == FLAG_BREAKDOWN)
            return fail(HISQ_ERR_BREAKDOWN, "multi-shift CG breakdown");
    }
    if (!refine) {
        // the Krylov iterates as they are: each shift's FP64 true residual
        hisq_status result = HISQ_OK;
        for (int k = 0; k < nshift; ++k) {
            double r2 = 0.0;
            if (bnorm2 > 0.0 &&
                (s = S.true_residual(shifts[k], b, x[k], S.at<void>(L.r), &r2)) != HISQ_OK)
                return s;
            const double rel = bnorm2 > 0.0 ? std::sqrt(r2 / bnorm2) : 0.0;
            if (!(rel <= tol[k]) && result == HISQ_OK)
                result = HISQ_ERR_NOT_CONVERGED;
            if (info)
                info[k] = hisq_solve_info{krylov_iters[k], 0, rel, now_s() - t0, krylov_iters[k], 0};
        }
        if (result != HISQ_OK)
            fail(result, "a shift's Krylov iterate is above its tolerance (no refinement requested)");
        return result;
    }
    // refinement: every shift to its own FP64 true residual, the shifts as the
    // columns of one multi-RHS CG (groups of up to HISQ_MAX_RHS), each column
    // with its own shift and tolerance, starting from its x_k
    hisq_status result = HISQ_OK;
    int kmax = 0;
    for (int k = 0; k < nshift; ++k)
        kmax = std::max(kmax, krylov_iters[k]);
    const int group = std::min(nshift, (int)HISQ_MAX_RHS);
    for (int k0 = 0; k0 < nshift; k0 += group) {
        const int n = std::min(group, nshift - k0);
        Columns C{};
        for (int j = 0; j < n; ++j) {
            C.b[j] = b;
            C.x[j] = x[k0 + j];
            C.sigma[j] = shifts[k0 + j];
            C.tol[j] = tol[k0 + j];
        }
        std::vector<hisq_solve_info> one(n);
        const int left = std::max(1, max_iter - kmax);
        hisq_status rs = run_cg(S, C, n, left, delta, one.data(), &krylov_iters[k0]);
        if (rs == HISQ_ERR_DEVICE || rs == HISQ_ERR_INVALID_ARG)
            return rs;
        if (rs == HISQ_ERR_BREAKDOWN)
            result = rs;
        else if (rs == HISQ_ERR_NOT_CONVERGED && result == HISQ_OK)
            result = rs;
        if (info)
            for (int j = 0; j < n; ++j) {
                info[k0 + j] = one[j];
                info[k0 + j].seconds = now_s() - t0;
            }
    }
    if (result != HISQ_OK)
        fail(result, result == HISQ_ERR_BREAKDOWN ? "multi-shift refinement breakdown"
                                                  : "a shift did not reach its tolerance");
    return result;
}

hisq_status setup_solver(Solver &S, hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                         const void *links_inner, hisq_prec inner, int nrhs, int nshift, void *ws, size_t ws_bytes,
                         hipStream_t st) {
    S.ctx = ctx;
    S.g = make_geom(*lat);
    S.st = st;
    S.mass = mass;
    S.links64 = static_cast<const char *>(links_f64);
    S.lp_in = inner;
    S.links_in = inner == HISQ_FP64 ? S.links64 : static_cast<const char *>(links_inner);
    S.L = make_layout(S.g, inner, nrhs, nshift);
    if (ws_bytes < S.L.total)
        return fail(HISQ_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, S.L.total);
    S.ws = static_cast<char *>(ws);
    S.shape64 = pick_shape(ctx, S.g, HISQ_FP64, HISQ_FP64, 1);
    S.shape64m = nrhs > 1 ? pick_shape(ctx, S.g, HISQ_FP64, HISQ_FP64, nrhs) : S.shape64;
    S.shape_in = pick_shape(ctx, S.g, S.lp_in, S.L.fs, nrhs);
    // chunk length: ~1 ms of iterations, 8 .. 64
    const double bytes_per_iter = 2.0 * (double)S.g.vh * 16 * link_matrix_bytes(inner);
    const double est_us = bytes_per_iter / 5.0e6 + 12.0;
    S.iter_us = est_us;
    S.chunk = std::max(8, std::min(64, (int)(1000.0 / est_us)));
    return HISQ_OK;
}

hisq_status check_solver_args(const hisq_lattice *lat, double mass, const void *links_f64, const void *links_inner,
                              hisq_prec inner, const void *ws) {
    hisq_status s = check_lattice(lat);
    if (s == HISQ_OK) s = check_prec(inner);
    if (s == HISQ_OK) s = check_ptr(links_f64, "links_f64");
    if (s == HISQ_OK && inner != HISQ_FP64) s = check_ptr(links_inner, "links_inner");
    if (s == HISQ_OK) s = check_ptr(ws, "ws");
    if (s == HISQ_OK && (!std::isfinite(mass) || mass * mass <= 0.0))
        s = fail(HISQ_ERR_INVALID_ARG, "mass^2 must be positive and finite (mass = %g)", mass);
    return s;
}

}  // namespace hisq

using namespace hisq;

extern "C" {

size_t hisq_cg_workspace_bytes(const hisq_lattice *lat, hisq_prec inner, int32_t nrhs, int32_t nshift) {
    if (check_lattice(lat) != HISQ_OK || check_prec(inner) != HISQ_OK)
        return 0;
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS || nshift < 0 || nshift > MAX_SHIFTS)
        return 0;
    return cg_workspace_bytes(make_geom(*lat), inner, nrhs, nshift);
}

hisq_status hisq_cg(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                    const void *links_inner, hisq_prec inner, int32_t nrhs, const void *b, void *x, double tol,
                    int32_t max_iter, void *ws, size_t ws_bytes, hisq_solve_info *info, void *stream) {
    hisq_status s = check_solver_args(lat, mass, links_f64, links_inner, inner, ws);
    if (s == HISQ_OK) s = check_nrhs(nrhs);
    if (s == HISQ_OK) s = check_ptr(b, "b");
    if (s == HISQ_OK) s = check_ptr(x, "x");
    if (s == HISQ_OK && !(tol > 0.0 && tol < 1.0))
        s = fail(HISQ_ERR_INVALID_ARG, "tol = %g must be in (0, 1)", tol);
    if (s == HISQ_OK && max_iter < 1)
        s = fail(HISQ_ERR_INVALID_ARG, "max_iter = %d must be >= 1", max_iter);
    if (s == HISQ_OK && b == x)
        s = fail(HISQ_ERR_INVALID_ARG, "b and x must not alias");
    if (s == HISQ_OK) s = set_device(ctx);
    if (s != HISQ_OK)
        return s;
    StreamGuard sg;
    hipError_t e = sg.init(static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return device_fail(e, "stream setup");
    Solver S;
    if ((s = setup_solver(S, ctx, lat, mass, links_f64, links_inner, inner, nrhs, 0, ws, ws_bytes, sg.own)) !=
        HISQ_OK)
        return s;
    // reliable updates whenever the iterated residual fell by 10x (reduced
    // precision); FP64 CG checks the true residual at convergence only
    const double delta = field_prec_of(inner) == HISQ_FP64 ? 0.0 : RELIABLE_DELTA;
    Columns C{};
    const size_t c64 = field_bytes(S.g, HISQ_FP64, 1);
    for (int j = 0; j < nrhs; ++j) {
        C.b[j] = static_cast<const char *>(b) + j * c64;
        C.x[j] = static_cast<char *>(x) + j * c64;
        C.sigma[j] = 0.0;
        C.tol[j] = tol;
    }
    return run_cg(S, C, nrhs, max_iter, delta, info, nullptr);
}

hisq_status hisq_chiral_condensate(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                                   const void *links_inner, hisq_prec inner, int32_t nnoise, const void *noise,
                                   void *x, double tol, int32_t max_iter, void *ws, size_t ws_bytes,
                                   double *samples, double *pbp, double *err, hisq_solve_info *info, void *stream) {
    hisq_status s = check_solver_args(lat, mass, links_f64, links_inner, inner, ws);
    if (s == HISQ_OK && nnoise < 1)
        s = fail(HISQ_ERR_INVALID_ARG, "nnoise = %d must be >= 1", nnoise);
    if (s == HISQ_OK) s = check_ptr(noise, "noise");
    if (s == HISQ_OK) s = check_ptr(x, "x");
    if (s == HISQ_OK) s = check_ptr(pbp, "pbp");
    if (s == HISQ_OK && noise == x)
        s = fail(HISQ_ERR_INVALID_ARG, "noise and x must not alias");
    if (s != HISQ_OK)
        return s;
    const Geom g = make_geom(*lat);
    const int group = std::min<int>(nnoise, HISQ_MAX_RHS);
    const Layout L = make_layout(g, inner, group, 0);
    if (ws_bytes < L.total)
        return fail(HISQ_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, L.total);
    const size_t fb = field_bytes(g, HISQ_FP64, 1);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    double *partials = reinterpret_cast<double *>(static_cast<char *>(ws) + L.partials);
    double *dots_d = reinterpret_cast<double *>(static_cast<char *>(ws) + L.scal) + 32;
    std::vector<double> dots(nnoise);
    std::vector<hisq_solve_info> inf(HISQ_MAX_RHS);
    hisq_status worst = HISQ_OK;
    for (int j0 = 0; j0 < nnoise; j0 += group) {
        const int n = std::min(group, nnoise - j0);
        const char *b = static_cast<const char *>(noise) + (size_t)j0 * fb;
        char *xj = static_cast<char *>(x) + (size_t)j0 * fb;
        hipError_t e = hipMemsetAsync(xj, 0, (size_t)n * fb, st);
        if (e != hipSuccess)
            return device_fail(e, "condensate: zero x");
        s = hisq_cg(ctx, lat, mass, links_f64, links_inner, inner, n, b, xj, tol, max_iter, ws, ws_bytes,
                    inf.data(), stream);
        if (s != HISQ_OK && s != HISQ_ERR_NOT_CONVERGED && s != HISQ_ERR_BREAKDOWN)
            return s;
        if (s != HISQ_OK && worst == HISQ_OK)
            worst = s;
        if (info)
            for (int k = 0; k < n; ++k)
                info[j0 + k] = inf[k];
        e = launch_dot_re(g.vh, n, b, xj, partials, dots_d, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dots.data() + j0, dots_d, sizeof(double) * n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return device_fail(e, "condensate: dot products");
    }
    // s_i = (2 m / V) Re <eta_i, M_e^-1 eta_i>; mean and standard error
    const double scale = 2.0 * mass / (2.0 * (double)g.vh);
    double mean = 0.0;
    for (int k = 0; k < nnoise; ++k) {
        const double v = scale * dots[k];
        if (samples)
            samples[k] = v;
        mean += v;
    }
    mean /= nnoise;
    double var = 0.0;
    for (int k = 0; k < nnoise; ++k) {
        const double d = scale * dots[k] - mean;
        var += d * d;
    }
    *pbp = mean;
    if (err)
        *err = nnoise > 1 ? std::sqrt(var / (nnoise - 1) / nnoise) : std::nan("");
    return worst;
}

static hisq_status multishift_entry(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                                    const void *links_inner, hisq_prec inner, int32_t nshift, const double *shifts,
                                    const void *b, void *const *x, const double *tol, int32_t max_iter, void *ws,
                                    size_t ws_bytes, hisq_solve_info *info, void *stream, bool refine) {
    hisq_status s = check_solver_args(lat, mass, links_f64, links_inner, inner, ws);
    if (s == HISQ_OK && (nshift < 1 || nshift > MAX_SHIFTS))
        s = fail(HISQ_ERR_INVALID_ARG, "nshift = %d outside [1, %d]", nshift, MAX_SHIFTS);
    if (s == HISQ_OK) s = check_ptr(shifts, "shifts");
    if (s == HISQ_OK) s = check_ptr(tol, "tol");
    if (s == HISQ_OK) s = check_ptr(b, "b");
    if (s == HISQ_OK) s = check_ptr(x, "x");
    if (s == HISQ_OK && max_iter < 1)
        s = fail(HISQ_ERR_INVALID_ARG, "max_iter = %d must be >= 1", max_iter);
    for (int k = 0; s == HISQ_OK && k < nshift; ++k) {
        if (!std::isfinite(shifts[k]) || mass * mass + shifts[k] <= 0.0)
            s = fail(HISQ_ERR_INVALID_ARG, "m^2 + shift[%d] = %g must be positive", k, mass * mass + shifts[k]);
        else if (!(tol[k] > 0.0 && tol[k] < 1.0))
            s = fail(HISQ_ERR_INVALID_ARG, "tol[%d] = %g must be in (0, 1)", k, tol[k]);
        else if (!x[k] || x[k] == b)
            s = fail(HISQ_ERR_INVALID_ARG, "x[%d] is NULL or aliases b", k);
        for (int j = 0; s == HISQ_OK && j < k; ++j)
            if (x[j] == x[k])
                s = fail(HISQ_ERR_INVALID_ARG, "x[%d] and x[%d] alias", j, k);
    }
    if (s == HISQ_OK) s = set_device(ctx);
    if (s != HISQ_OK)
        return s;
    StreamGuard sg;
    hipError_t e = sg.init(static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return device_fail(e, "stream setup");
    Solver S;
    if ((s = setup_solver(S, ctx, lat, mass, links_f64, links_inner, inner, 1, nshift, ws, ws_bytes, sg.own)) !=
        HISQ_OK)
        return s;
    const double delta = field_prec_of(inner) == HISQ_FP64 ? 0.0 : RELIABLE_DELTA;
    return run_multishift(S, nshift, shifts, b, x, tol, max_iter, delta, info, refine);
}

hisq_status hisq_multishift_cg(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                               const void *links_inner, hisq_prec inner, int32_t nshift, const double *shifts,
                               const void *b, void *const *x, const double *tol, int32_t max_iter, void *ws,
                               size_t ws_bytes, hisq_solve_info *info, void *stream) {
    return multishift_entry(ctx, lat, mass, links_f64, links_inner, inner, nshift, shifts, b, x, tol, max_iter, ws,
                            ws_bytes, info, stream, true);
}

hisq_status hisq_multishift_krylov(hisq_context *ctx, const hisq_lattice *lat, double mass, const void *links_f64,
                                   const void *links_inner, hisq_prec inner, int32_t nshift, const double *shifts,
                                   const void *b, void *const *x, const double *tol, int32_t max_iter, void *ws,
                                   size_t ws_bytes, hisq_solve_info *info, void *stream) {
    return multishift_entry(ctx, lat, mass, links_f64, links_inner, inner, nshift, shifts, b, x, tol, max_iter, ws,
                            ws_bytes, info, stream, false);
}

}  // extern "C"
