// ffmg_batch.hip -- many independent solves (incoming directions, energies,
// grid sizes) advanced together: one launch per kernel for all instances, the
// refinement step of the whole batch captured once in a HIP graph and replayed
// until every instance has met its stopping test on the device.
//
// Instance i is (operator hs[i], incoming direction eta_i); operators may be
// shared.  Each instance's V-cycle is the sequence of the single-instance
// fused 2D path (pre-smoothing, residual + restriction, the one-workgroup LDS
// tail, interpolation + post-smoothing) on its own workspace.  Levels are
// aligned at the coarse end: at step s of the down-sweep an instance with D
// levels above the tail works on its level s - (Dmax - D), so all tails run in
// one launch of one workgroup per instance, and every launch's tiles are the
// concatenated tiles of the instances active at that step.  Every kernel keeps
// the per-instance block structure of the single path, so each instance's
// iterates and residual norms are bit for bit those of mg_solve.
//
// The FP64 iterate alternates between the caller's u and a workspace buffer;
// the graph holds two refinement steps (u -> t, t -> u) so that it is the
// same on every replay.  A converged instance's stop flag makes its later
// launches exit at once.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <vector>

#include "ffmg_handle.hpp"

namespace ffmg {

struct BatchInst {
    ffmg_handle *op = nullptr;
    int D = 0;                            // levels above the tail (tail starts at level D)
    cd *t = nullptr;                      // the other buffer of the FP64 iterate
    cd *f = nullptr;                      // the plane wave's per-axis factors (b = q u_in is never stored)
    std::vector<cf *> u32, b32, t32, r32; // FP32 cycle: levels 0..D (t32, r32: 0..D-1)
    double *parts = nullptr;
    SolveCtl *ctl = nullptr;
    int nb_norm = 0, nb_res = 0, tiles_res = 0, ref_tiles = 0, ref_tx = 0;
};

struct Batch {
    std::vector<uint64_t> key;
    std::vector<BatchInst> inst;
    int count = 0, Dmax = 0, nu1 = 0, nu2 = 0, inner = 0;
    int variant = 0, th_smooth = 8, th_srr = 16;   // FFMG_TUNE_BATCH and its tile heights
    int fmg = 0;                          // V-cycles per level of the full multigrid start (0: u = 0)
    size_t tail_lds = 0;
    int max_nb_norm = 0, max_nb_res = 0, ref_ntiles = 0, max_m = 0;
    int last_steps = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t fmg_graph = nullptr;       // the full multigrid start of every instance
    hipGraphExec_t fmg_exec = nullptr;
    XferJob *d_xfin = nullptr;            // its last transfer, into the caller's u (written per call)
    std::vector<XferJob> xfin;
    size_t max_n0 = 0;
    std::vector<void *> allocs;
    InitJob *d_init = nullptr;
    CtlJob *d_ctl0 = nullptr, *d_ctl = nullptr;
    RefineJob *d_refA = nullptr, *d_refB = nullptr;
    int *d_ref_tile_job = nullptr;
    FinishJob *d_finish = nullptr;
    int *d_ndone = nullptr;
    int *h_ndone = nullptr;               // pinned
    SolveCtl *h_ctls = nullptr;           // pinned
    std::vector<InitJob> init;
    std::vector<RefineJob> refA, refB;
    std::vector<FinishJob> fin;

    hipError_t alloc(void **p, size_t bytes)
    {
        hipError_t e = hipMalloc(p, bytes ? bytes : 16);
        if (e == hipSuccess) allocs.push_back(*p);
        return e;
    }
    ~Batch()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (fmg_exec) (void)hipGraphExecDestroy(fmg_exec);
        if (fmg_graph) (void)hipGraphDestroy(fmg_graph);
        for (void *p : allocs) (void)hipFree(p);
        if (h_ndone) (void)hipHostFree(h_ndone);
        if (h_ctls) (void)hipHostFree(h_ctls);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

void batch_destroy(Batch *b) { delete b; }

namespace {

#define BCHK(x)                                                                                                     \
    do {                                                                                                            \
        hipError_t e_ = (x);                                                                                        \
        if (e_ != hipSuccess)                                                                                       \
            return fail(h0, e_ == hipErrorOutOfMemory ? FFMG_ENOMEM : FFMG_EDEVICE, "%s: %s (%s:%d)", #x,         \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                                 \
    } while (0)

// Host-side lists of the level launches of one FP32 V-cycle; uploaded once.
struct LaunchRec {
    int kind;            // 0 smooth, 1 resid+restrict, 2 tail, 3 one-pass pre-smoothing + resid + restrict,
                         // 4 grid transfer of the start, 5 the tail's full multigrid start
    int ns = 0;          // smooth: sweeps in this launch; transfer: its kind; tail start: cycles per level
    bool zero = false, prol = false;
    size_t job_off = 0;  // index into the typed job array
    size_t tj_off = 0;   // index into tile_job
    int ntiles = 0;      // tiles (or jobs for the tail and the transfers)
    size_t max_n = 0;    // transfer: largest output grid
};

struct Plan {
    std::vector<SmoothJob<float>> sj;
    std::vector<RRJob<float>> rj;
    std::vector<SRRJob<float>> srj;
    std::vector<TailJob<float>> tj;
    std::vector<int> tile_job;
    std::vector<LaunchRec> recs;   // one inner V-cycle with the finest guess nonzero
    std::vector<LaunchRec> recs0;  // the first inner V-cycle (zero finest guess)
    std::vector<XferJob> xj;
    std::vector<TailJob<float>> tfj;
    std::vector<LaunchRec> fmg;    // the full multigrid start up to level 1
};

// Append one smooth launch over the given (instance, level, src, dst, ec, zero) entries.
struct SmoothEntry {
    int i, l;
    const cf *src;
    cf *dst;
    const cf *ec;
};

void add_smooth(Plan &pl, std::vector<LaunchRec> &out, Batch &B, const std::vector<SmoothEntry> &es, int ns,
                bool zero, bool prol)
{
    if (es.empty()) return;
    LaunchRec r;
    r.kind = 0;
    r.ns = ns;
    r.zero = zero;
    r.prol = prol;
    r.job_off = pl.sj.size();
    r.tj_off = pl.tile_job.size();
    int tot = 0;
    for (const SmoothEntry &e : es) {
        BatchInst &I = B.inst[e.i];
        Level &lv = I.op->L[e.l];
        int tx;
        int nt = smooth2d_tiles<float>(lv.g, &tx, B.th_smooth);
        SmoothJob<float> j;
        j.u = e.src;
        j.ec = e.ec;
        j.b = I.b32[e.l];
        j.q = lv.q32;
        j.out = e.dst;
        j.P = lv.P32;
        j.tiles_x = tx;
        j.tile0 = tot;
        j.stop = &I.ctl->done;
        int jid = (int)(pl.sj.size() - r.job_off);
        pl.sj.push_back(j);
        for (int t = 0; t < nt; ++t) pl.tile_job.push_back(jid);
        tot += nt;
    }
    r.ntiles = tot;
    out.push_back(r);
}

// Append one one-pass pre-smoothing launch (two sweeps u32 -> t32, residual
// and restriction into b32[l + 1]) over the (instance, level) entries.
void add_srr(Plan &pl, std::vector<LaunchRec> &out, Batch &B, const std::vector<std::pair<int, int>> &es, bool zero)
{
    if (es.empty()) return;
    LaunchRec r;
    r.kind = 3;
    r.zero = zero;
    r.job_off = pl.srj.size();
    r.tj_off = pl.tile_job.size();
    int tot = 0;
    for (const auto &e : es) {
        BatchInst &I = B.inst[e.first];
        const int l = e.second;
        Level &lv = I.op->L[l];
        int tx;
        int nt = smooth_rr2d_tiles<float>(lv.g, &tx, B.th_srr);
        SRRJob<float> j;
        j.u = I.u32[l];
        j.b = I.b32[l];
        j.q = lv.q32;
        j.out = I.t32[l];
        j.bc = I.b32[l + 1];
        j.P = lv.P32;
        j.tiles_x = tx;
        j.tile0 = tot;
        j.stop = &I.ctl->done;
        int jid = (int)(pl.srj.size() - r.job_off);
        pl.srj.push_back(j);
        for (int t = 0; t < nt; ++t) pl.tile_job.push_back(jid);
        tot += nt;
    }
    r.ntiles = tot;
    out.push_back(r);
}

// The launches of one V-cycle.  S = 0: the inner V-cycle of a refinement
// step from each instance's finest level (first: zero guess there).  S >= 1:
// a V-cycle of the full multigrid start rooted at step S, i.e. at level
// S - (Dmax - D) >= 1 of each instance that has that level, with the
// interpolated coarser solution as its guess.
void build_cycle(Plan &pl, std::vector<LaunchRec> &out, Batch &B, bool first, int S = 0)
{
    const int Dmax = B.Dmax, n = B.count;
    auto root_of = [&](int i) { return S == 0 ? 0 : S - (Dmax - B.inst[i].D); };
    auto in_cycle = [&](int i) { return S == 0 || root_of(i) >= 1; };
    auto level_of = [&](int i, int s) {   // < 0: not active at step s
        const int l = s - (Dmax - B.inst[i].D);
        return (in_cycle(i) && l >= root_of(i)) ? l : -1;
    };
    // down-sweep
    for (int s = S; s < Dmax; ++s) {
        if (B.nu1 == 2) {
            // two sweeps, residual and restriction in one pass: u -> t, b_c
            std::vector<std::pair<int, int>> ez, enz;
            for (int i = 0; i < n; ++i) {
                const int l = level_of(i, s);
                if (l < 0) continue;
                ((l > root_of(i) || first) ? ez : enz).push_back({i, l});
            }
            add_srr(pl, out, B, ez, true);
            add_srr(pl, out, B, enz, false);
            continue;
        }
        // pre-smoothing chain: nu1 sweeps, two per launch, u -> t (tmp r)
        const int nk = (B.nu1 + 1) / 2;
        int left = B.nu1;
        for (int kk = 0; kk < nk; ++kk) {
            const int ns = left >= 2 ? 2 : 1;
            left -= ns;
            std::vector<SmoothEntry> ez, enz;
            for (int i = 0; i < n; ++i) {
                const int l = level_of(i, s);
                if (l < 0) continue;
                BatchInst &I = B.inst[i];
                cf *dst = ((nk - 1 - kk) % 2 == 0) ? I.t32[l] : I.r32[l];
                const cf *src;
                if (kk == 0) src = I.u32[l];
                else src = ((nk - 1 - (kk - 1)) % 2 == 0) ? I.t32[l] : I.r32[l];
                const bool zero = (kk == 0) && (l > root_of(i) || first);
                (zero ? ez : enz).push_back(SmoothEntry{i, l, src, dst, nullptr});
            }
            add_smooth(pl, out, B, ez, ns, true, false);
            add_smooth(pl, out, B, enz, ns, false, false);
        }
        // residual + restriction: t -> b32[l + 1]
        LaunchRec r;
        r.kind = 1;
        r.job_off = pl.rj.size();
        r.tj_off = pl.tile_job.size();
        int tot = 0;
        for (int i = 0; i < n; ++i) {
            const int l = level_of(i, s);
            if (l < 0) continue;
            BatchInst &I = B.inst[i];
            Level &lv = I.op->L[l];
            int ctx;
            int nt = resid_restrict2d_tiles(lv.g, &ctx);
            RRJob<float> j;
            j.u = I.t32[l];
            j.b = I.b32[l];
            j.q = lv.q32;
            j.bc = I.b32[l + 1];
            j.P = lv.P32;
            j.ctiles_x = ctx;
            j.tile0 = tot;
            j.stop = &I.ctl->done;
            int jid = (int)(pl.rj.size() - r.job_off);
            pl.rj.push_back(j);
            for (int t = 0; t < nt; ++t) pl.tile_job.push_back(jid);
            tot += nt;
        }
        r.ntiles = tot;
        if (tot > 0) out.push_back(r);
    }
    // the coarse end of every instance in one launch
    {
        LaunchRec r;
        r.kind = 2;
        r.job_off = pl.tj.size();
        r.ntiles = 0;
        for (int i = 0; i < n; ++i) {
            if (!in_cycle(i)) continue;
            ++r.ntiles;
            BatchInst &I = B.inst[i];
            TailJob<float> j;
            j.tp = I.op->tail32;
            j.b_top = I.b32[I.D];
            j.u_top = I.u32[I.D];
            j.stop = &I.ctl->done;
            pl.tj.push_back(j);
        }
        out.push_back(r);
    }
    // up-sweep: interpolation + post-smoothing chain t -> u (tmp r)
    for (int s = Dmax - 1; s >= S; --s) {
        const int nk = (B.nu2 + 1) / 2;
        int left = B.nu2;
        for (int kk = 0; kk < nk; ++kk) {
            const int ns = left >= 2 ? 2 : 1;
            left -= ns;
            std::vector<SmoothEntry> es;
            for (int i = 0; i < n; ++i) {
                const int l = level_of(i, s);
                if (l < 0) continue;
                BatchInst &I = B.inst[i];
                cf *dst = ((nk - 1 - kk) % 2 == 0) ? I.u32[l] : I.r32[l];
                const cf *src;
                if (kk == 0) src = I.t32[l];
                else src = ((nk - 1 - (kk - 1)) % 2 == 0) ? I.u32[l] : I.r32[l];
                es.push_back(SmoothEntry{i, l, src, dst, kk == 0 ? I.u32[l + 1] : nullptr});
            }
            add_smooth(pl, out, B, es, ns, false, kk == 0);
        }
    }
}

// One transfer launch of the start over the given jobs.
void add_xfer(Plan &pl, std::vector<LaunchRec> &out, int kind, const std::vector<XferJob> &js)
{
    if (js.empty()) return;
    LaunchRec r;
    r.kind = 4;
    r.ns = kind;
    r.job_off = pl.xj.size();
    r.ntiles = (int)js.size();
    for (const XferJob &j : js) {
        const size_t n = (kind <= 1) ? (size_t)j.mxc * j.myc : (size_t)j.mxf * j.myf;
        r.max_n = std::max(r.max_n, n);
        pl.xj.push_back(j);
    }
    out.push_back(r);
}

XferJob xfer_job(const BatchInst &I, int l, const void *src, void *dst, bool f64_end)
{
    const LevelGeom &f = I.op->L[l].g, &c = I.op->L[l + 1].g;
    XferJob j;
    j.src = src;
    j.dst = dst;
    j.qf = nullptr;
    j.pwf = nullptr;
    j.mxf = f.m[0];
    j.myf = f.m[1];
    j.mxc = c.m[0];
    j.myc = c.m[1];
    j.bnorm2 = f64_end ? &I.ctl->b2 : nullptr;
    j.inv_sqN = 1.0 / sqrt((double)I.op->L[0].g.N());
    j.stop = &I.ctl->done;
    return j;
}

// The full multigrid start of every instance in the order of the
// single-instance start: the finest right-hand side (scaled to unit RMS)
// injected level by level down to the first tail level, the tails' nested
// iteration, then level by level finest-ward the interpolated coarser
// solution and k V-cycles, down to level 1; the last interpolation (into
// the caller's FP64 u) is added per call.
void build_fmg(Plan &pl, Batch &B, int k)
{
    const int Dmax = B.Dmax, n = B.count;
    std::vector<XferJob> js;
    for (int i = 0; i < n; ++i) {
        BatchInst &I = B.inst[i];
        XferJob j = xfer_job(I, 0, nullptr, I.b32[1], true);   // b = q u_in formed at the injected points
        j.qf = I.op->L[0].q;
        j.pwf = I.f;
        js.push_back(j);
    }
    add_xfer(pl, pl.fmg, 0, js);
    for (int s = 1; s < Dmax; ++s) {
        js.clear();
        for (int i = 0; i < n; ++i) {
            BatchInst &I = B.inst[i];
            const int l = s - (Dmax - I.D);
            if (l >= 1 && l < I.D) js.push_back(xfer_job(I, l, I.b32[l], I.b32[l + 1], false));
        }
        add_xfer(pl, pl.fmg, 1, js);
    }
    LaunchRec r;
    r.kind = 5;
    r.ns = k;
    r.job_off = pl.tfj.size();
    r.ntiles = n;
    for (int i = 0; i < n; ++i) {
        BatchInst &I = B.inst[i];
        TailJob<float> j;
        j.tp = I.op->tail32;
        j.b_top = I.b32[I.D];
        j.u_top = I.u32[I.D];
        j.stop = &I.ctl->done;
        pl.tfj.push_back(j);
    }
    pl.fmg.push_back(r);
    for (int S = Dmax - 1; S >= 1; --S) {
        js.clear();
        for (int i = 0; i < n; ++i) {
            BatchInst &I = B.inst[i];
            const int l = S - (Dmax - I.D);
            if (l >= 1) js.push_back(xfer_job(I, l, I.u32[l + 1], I.u32[l], false));
        }
        add_xfer(pl, pl.fmg, 2, js);
        std::vector<LaunchRec> cyc;
        build_cycle(pl, cyc, B, false, S);
        for (int c = 0; c < k; ++c) pl.fmg.insert(pl.fmg.end(), cyc.begin(), cyc.end());
    }
}

template <typename J>
hipError_t upload(Batch &B, J **d, const std::vector<J> &h)
{
    hipError_t e = B.alloc((void **)d, h.size() * sizeof(J));
    if (e != hipSuccess) return e;
    return hipMemcpy(*d, h.data(), h.size() * sizeof(J), hipMemcpyHostToDevice);
}

struct DevPlan {
    SmoothJob<float> *sj = nullptr;
    RRJob<float> *rj = nullptr;
    TailJob<float> *tj = nullptr, *tfj = nullptr;
    SRRJob<float> *srj = nullptr;
    XferJob *xj = nullptr;
    int *tile_job = nullptr;
};

void enqueue_cycle(const Batch &B, const std::vector<LaunchRec> &recs, const DevPlan &d)
{
    const SmoothJob<float> *sj = d.sj;
    const RRJob<float> *rj = d.rj;
    const TailJob<float> *tj = d.tj;
    const SRRJob<float> *srj = d.srj;
    const int *tile_job = d.tile_job;
    for (const LaunchRec &r : recs) {
        if (r.kind == 4)
            launch_xfer_batch(r.ns, d.xj + r.job_off, r.ntiles, r.max_n, B.stream);
        else if (r.kind == 5)
            launch_tail2d_fmg_batch<float>(d.tfj + r.job_off, r.ntiles, r.ns, B.tail_lds, B.stream);
        else if (r.kind == 3)
            launch_smooth_rr2d_batch<float>(r.zero, srj + r.job_off, tile_job + r.tj_off, r.ntiles, B.stream,
                                            B.th_srr);
        else if (r.kind == 0)
            launch_smooth2d_batch<float>(r.ns, r.zero, r.prol, sj + r.job_off, tile_job + r.tj_off, r.ntiles,
                                         B.stream, B.th_smooth);
        else if (r.kind == 1)
            launch_resid_restrict2d_batch<float>(rj + r.job_off, tile_job + r.tj_off, r.ntiles, B.stream);
        else
            launch_tail2d_batch<float>(tj + r.job_off, r.ntiles, B.tail_lds, B.stream);
    }
}

ffmg_status build_batch(ffmg_handle *const *hs, int count, Batch **out)
{
    ffmg_handle *h0 = hs[0];
    Batch *Bp = new Batch();
    Batch &B = *Bp;
    auto bail = [&](ffmg_status s) {
        delete Bp;
        return s;
    };
    B.count = count;
    B.variant = h0->batch_variant;
    batch_tiles(B.variant, &B.th_smooth, &B.th_srr);
    const ffmg_options &o0 = h0->opt;
    B.nu1 = o0.nu1;
    B.nu2 = o0.nu2;
    B.inner = o0.inner_cycles > 0 ? o0.inner_cycles : DEFAULT_INNER_CYCLES;
    B.fmg = o0.fmg_cycles;
    for (int i = 0; i < count; ++i) {
        ffmg_handle *h = hs[i];
        if (!h) return bail(fail(h0, FFMG_EINVAL, "hs[%d] is null", i));
        B.key.push_back(h->serial);
        const ffmg_options &o = h->opt;
        if (h->prob.dim != 2 || o.precision != FFMG_FP32_IR || o.tile_config != TILE_FUSED)
            return bail(fail(h0, FFMG_EINVAL,
                             "instance %d: batched solves need 2D operators set up with precision FP32_IR and the "
                             "fused kernels (tile_config 0)", i));
        if (o.fmg_cycles != o0.fmg_cycles || o.fmg_cycles < 0)
            return bail(fail(h0, FFMG_EINVAL, "instance %d: every operator needs the same fmg_cycles", i));
        if (o.nu1 != B.nu1 || o.nu2 != B.nu2 || o.nu1 < 1 || o.nu2 < 1 ||
            (o.nu_coarse != 0 && (o.nu_coarse != o.nu1 || o.nu_coarse != o.nu2)) ||
            (o.inner_cycles > 0 ? o.inner_cycles : DEFAULT_INNER_CYCLES) != B.inner || o.smoother != FFMG_SMOOTH_JACOBI)
            return bail(fail(h0, FFMG_EINVAL, "instance %d: every operator needs the same nu1, nu2 >= 1 and inner "
                                              "cycles", i));
        const TailParams<float> &tp = h->tail32, &t0 = h0->tail32;
        if (tp.nt < 2 || tp.nt != t0.nt || h->nc != h0->nc || h->tail_lds[1] != h0->tail_lds[1])
            return bail(fail(h0, FFMG_EINVAL, "instance %d: the coarse ends of the operators differ", i));
        for (int k = 0; k < tp.nt; ++k)
            if (tp.lv[k].mx != t0.lv[k].mx || tp.lv[k].my != t0.lv[k].my)
                return bail(fail(h0, FFMG_EINVAL, "instance %d: the coarse ends of the operators differ", i));
        BatchInst I;
        I.op = h;
        I.D = (int)h->L.size() - tp.nt;
        if (I.D < 1) return bail(fail(h0, FFMG_EINVAL, "instance %d: grid too small for a batched solve", i));
        B.Dmax = std::max(B.Dmax, I.D);
        B.inst.push_back(I);
    }
    B.tail_lds = h0->tail_lds[1];
    // workspaces
    for (BatchInst &I : B.inst) {
        const LevelGeom &g0 = I.op->L[0].g;
        const size_t N0 = g0.N();
        BCHK(B.alloc((void **)&I.t, N0 * sizeof(cd)));
        BCHK(B.alloc((void **)&I.f, (size_t)(g0.m[0] + g0.m[1]) * sizeof(cd)));
        B.max_m = std::max(B.max_m, std::max(g0.m[0], g0.m[1]));
        I.u32.assign(I.D + 1, nullptr);
        I.b32.assign(I.D + 1, nullptr);
        I.t32.assign(I.D, nullptr);
        I.r32.assign(I.D, nullptr);
        for (int l = 0; l <= I.D; ++l) {
            const size_t N = I.op->L[l].g.N();
            BCHK(B.alloc((void **)&I.u32[l], N * sizeof(cf)));
            BCHK(B.alloc((void **)&I.b32[l], N * sizeof(cf)));
            if (l < I.D) {
                BCHK(B.alloc((void **)&I.t32[l], N * sizeof(cf)));
                if (B.nu1 > 2 || B.nu2 > 2) BCHK(B.alloc((void **)&I.r32[l], N * sizeof(cf)));
            }
        }
        I.nb_norm = norm2_blocks(N0);
        I.nb_res = stencil_blocks(g0);
        int tx;
        I.ref_tiles = refine2d_tiles(g0, &tx);
        I.ref_tx = tx;
        const int np = std::max(std::max(I.nb_norm, I.nb_res), I.ref_tiles);
        BCHK(B.alloc((void **)&I.parts, (size_t)np * sizeof(double)));
        BCHK(B.alloc((void **)&I.ctl, sizeof(SolveCtl)));
        B.max_nb_norm = std::max(B.max_nb_norm, I.nb_norm);
        B.max_nb_res = std::max(B.max_nb_res, I.nb_res);
    }
    // static job tables
    Plan pl;
    build_cycle(pl, pl.recs0, B, true);
    build_cycle(pl, pl.recs, B, false);
    if (B.fmg > 0) build_fmg(pl, B, B.fmg);
    std::vector<CtlJob> c0, c1;
    std::vector<int> rtj;
    for (int i = 0; i < count; ++i) {
        BatchInst &I = B.inst[i];
        c0.push_back(CtlJob{I.ctl, I.parts, I.nb_res});
        c1.push_back(CtlJob{I.ctl, I.parts, I.ref_tiles});
        for (int t = 0; t < I.ref_tiles; ++t) rtj.push_back(i);
        B.ref_ntiles += I.ref_tiles;
    }
    DevPlan dp;
    BCHK(upload(B, &dp.sj, pl.sj));
    BCHK(upload(B, &dp.rj, pl.rj));
    BCHK(upload(B, &dp.tj, pl.tj));
    BCHK(upload(B, &dp.srj, pl.srj));
    BCHK(upload(B, &dp.tile_job, pl.tile_job));
    BCHK(upload(B, &dp.xj, pl.xj));
    BCHK(upload(B, &dp.tfj, pl.tfj));
    BCHK(upload(B, &B.d_ctl0, c0));
    BCHK(upload(B, &B.d_ctl, c1));
    BCHK(upload(B, &B.d_ref_tile_job, rtj));
    B.init.resize(count);
    B.refA.resize(count);
    B.refB.resize(count);
    B.fin.resize(count);
    BCHK(B.alloc((void **)&B.d_init, count * sizeof(InitJob)));
    BCHK(B.alloc((void **)&B.d_refA, count * sizeof(RefineJob)));
    BCHK(B.alloc((void **)&B.d_refB, count * sizeof(RefineJob)));
    BCHK(B.alloc((void **)&B.d_finish, count * sizeof(FinishJob)));
    BCHK(B.alloc((void **)&B.d_ndone, sizeof(int)));
    BCHK(B.alloc((void **)&B.d_xfin, count * sizeof(XferJob)));
    B.xfin.resize(count);
    for (int i = 0; i < count; ++i) {
        B.xfin[i] = xfer_job(B.inst[i], 0, B.inst[i].u32[1], nullptr, true);
        B.max_n0 = std::max(B.max_n0, B.inst[i].op->L[0].g.N());
    }
    BCHK(hipHostMalloc((void **)&B.h_ndone, sizeof(int), hipHostMallocDefault));
    BCHK(hipHostMalloc((void **)&B.h_ctls, count * sizeof(SolveCtl), hipHostMallocDefault));
    BCHK(hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking));
    // the tail kernels' LDS limit must be raised before capture
    launch_tail2d_batch<float>(nullptr, 0, 0, B.stream);
    launch_tail2d_fmg_batch<float>(nullptr, 0, 0, 0, B.stream);
    // the graph: two refinement steps (u -> t, t -> u) and the count of
    // finished instances
    BCHK(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal));
    for (int step = 0; step < 2; ++step) {
        for (int c = 0; c < B.inner; ++c)
            enqueue_cycle(B, c == 0 ? pl.recs0 : pl.recs, dp);
        launch_refine2d_batch(step == 0 ? B.d_refA : B.d_refB, B.d_ref_tile_job, B.ref_ntiles, B.stream);
        launch_ctl_update_batch(B.d_ctl, count, B.stream);
    }
    launch_count_done(B.d_ctl, count, B.d_ndone, B.stream);
    hipError_t ce = hipStreamEndCapture(B.stream, &B.graph);
    if (ce != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(h0, FFMG_EDEVICE, "graph capture failed: %s", hipGetErrorString(ce)));
    }
    BCHK(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    if (B.fmg > 0) {
        // the start: its static part, then the interpolation into the
        // caller's u from the job table written before each launch
        BCHK(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal));
        enqueue_cycle(B, pl.fmg, dp);
        launch_xfer_batch(3, B.d_xfin, count, B.max_n0, B.stream);
        ce = hipStreamEndCapture(B.stream, &B.fmg_graph);
        if (ce != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(h0, FFMG_EDEVICE, "graph capture failed: %s", hipGetErrorString(ce)));
        }
        BCHK(hipGraphInstantiate(&B.fmg_exec, B.fmg_graph, nullptr, nullptr, 0));
    }
    *out = Bp;
    return FFMG_OK;
}

}  // namespace
}  // namespace ffmg

using namespace ffmg;

extern "C" {

ffmg_status mg_solve_batched(ffmg_handle *const *hs, int count, const double *etas, void *const *u, double tol,
                             ffmg_solve_info *infos)
{
    if (!hs || count < 1 || !hs[0]) return FFMG_EINVAL;
    ffmg_handle *h0 = hs[0];
    if (!etas || !u) return fail(h0, FFMG_EINVAL, "null argument");
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(h0, FFMG_EINVAL, "tol must lie in (0, 1)");
    for (int i = 0; i < count; ++i) {
        if (!hs[i] || !u[i]) return fail(h0, FFMG_EINVAL, "hs[%d] or u[%d] is null", i, i);
        if (hs[i]->pend.active)
            return fail(h0, FFMG_EINVAL, "hs[%d] has a solve begun by mg_solve_begin pending", i);
        for (int k = 0; k < 3; ++k)
            if (!isfinite(etas[3 * i + k])) return fail(h0, FFMG_EINVAL, "eta of instance %d is not finite", i);
    }
    // the workspace and graph are cached on hs[0] for this list of handles
    std::vector<uint64_t> key;
    for (int i = 0; i < count; ++i) key.push_back(hs[i]->serial);
    if (!h0->batch || h0->batch->key != key || h0->batch->variant != h0->batch_variant) {
        if (h0->batch) batch_destroy(h0->batch);
        h0->batch = nullptr;
        TRY(build_batch(hs, count, &h0->batch));
    }
    Batch &B = *h0->batch;
    for (int i = 0; i < count; ++i) {
        ffmg_handle *h = hs[i];
        if (!(h->k0 > 0.0)) return fail(h0, FFMG_EINVAL, "instance %d: a plane wave needs E > 0", i);
        if (exponent_budget(h) > 700.0)
            return fail(h0, FFMG_ERANGE, "instance %d: exp(i k0 eta.z) overflows double on this box", i);
        BatchInst &I = B.inst[i];
        Level &l0 = h->L[0];
        const LevelGeom &g = l0.g;
        InitJob &J = B.init[i];
        J.q = l0.q;
        J.u = (cd *)u[i];
        J.f = I.f;
        J.r32 = I.b32[0];
        J.ctl = I.ctl;
        J.partial = I.parts;
        J.P = l0.P64;
        J.g = g;
        for (int k = 0; k < 3; ++k) J.eta[k] = etas[3 * i + k];
        J.ar_s = -(h->k0 * sin(h->prob.gamma));
        J.ai_s = h->k0 * cos(h->prob.gamma);
        J.tol = tol;
        J.inv_sqN = 1.0 / sqrt((double)g.N());
        J.max_cycles = h->opt.max_cycles;
        J.nb_norm = I.nb_norm;
        J.nb_res = I.nb_res;
        int snb, stx;
        stencil_grid2d(g, &snb, &stx);
        J.tiles_x = stx;
        RefineJob R;
        R.d = I.u32[0];
        R.b = nullptr;   // the plane wave's q u_in from I.f
        R.f = I.f;
        R.q = l0.q;
        R.r32 = I.b32[0];
        R.ctl = I.ctl;
        R.P = l0.P64;
        R.tiles_x = I.ref_tx;
        R.ntiles = I.ref_tiles;
        R.partial = I.parts;
        R.stop = &I.ctl->done;
        int t0 = 0;
        for (int k = 0; k < i; ++k) t0 += B.inst[k].ref_tiles;
        R.tile0 = t0;
        R.u = (const cd *)u[i];
        R.u_out = I.t;
        B.refA[i] = R;
        R.u = I.t;
        R.u_out = (cd *)u[i];
        B.refB[i] = R;
        B.fin[i] = FinishJob{I.t, (cd *)u[i], I.ctl, g.N()};
        B.xfin[i].dst = u[i];
    }
    hipEvent_t e0, e1, ein;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    BCHK(hipEventCreate(&ein));
    // order after the caller's stream (the RHS and u of the caller's work)
    BCHK(hipEventRecord(ein, h0->stream));
    BCHK(hipStreamWaitEvent(B.stream, ein, 0));
    BCHK(hipMemcpyAsync(B.d_init, B.init.data(), count * sizeof(InitJob), hipMemcpyHostToDevice, B.stream));
    BCHK(hipMemcpyAsync(B.d_refA, B.refA.data(), count * sizeof(RefineJob), hipMemcpyHostToDevice, B.stream));
    BCHK(hipMemcpyAsync(B.d_refB, B.refB.data(), count * sizeof(RefineJob), hipMemcpyHostToDevice, B.stream));
    BCHK(hipMemcpyAsync(B.d_finish, B.fin.data(), count * sizeof(FinishJob), hipMemcpyHostToDevice, B.stream));
    if (B.fmg > 0)
        BCHK(hipMemcpyAsync(B.d_xfin, B.xfin.data(), count * sizeof(XferJob), hipMemcpyHostToDevice, B.stream));
    BCHK(hipEventRecord(e0, B.stream));
    launch_init_batch(B.d_init, count, B.max_nb_norm, B.max_m, B.fmg == 0, B.stream);
    if (B.fmg > 0) BCHK(hipGraphLaunch(B.fmg_exec, B.stream));
    launch_init_resid_batch(B.d_init, count, B.max_nb_res, B.stream);
    launch_ctl_update_batch(B.d_ctl0, count, B.stream);
    BCHK(hipGetLastError());
    int maxc = 0;
    for (int i = 0; i < count; ++i) maxc = std::max(maxc, hs[i]->opt.max_cycles);
    const int max_replays = (maxc + 1) / 2 + 1;
    int replays = 0;
    int batch = B.last_steps > 0 ? (B.last_steps + 1) / 2 : 2;
    for (;;) {
        int nb = std::min(batch, max_replays - replays);
        for (int r = 0; r < nb; ++r) BCHK(hipGraphLaunch(B.exec, B.stream));
        replays += nb;
        BCHK(hipMemcpyAsync(B.h_ndone, B.d_ndone, sizeof(int), hipMemcpyDeviceToHost, B.stream));
        BCHK(hipStreamSynchronize(B.stream));
        if (*B.h_ndone >= count || replays >= max_replays) break;
        batch = 1;
    }
    launch_finish_batch(B.d_finish, count, B.stream);
    BCHK(hipEventRecord(e1, B.stream));
    for (int i = 0; i < count; ++i)
        BCHK(hipMemcpyAsync(B.h_ctls + i, B.inst[i].ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, B.stream));
    BCHK(hipStreamSynchronize(B.stream));
    // the caller's stream continues after the batch
    BCHK(hipEventRecord(ein, B.stream));
    BCHK(hipStreamWaitEvent(h0->stream, ein, 0));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(ein);
    ffmg_status worst = FFMG_OK;
    int kmax = 0;
    for (int i = 0; i < count; ++i) {
        const SolveCtl &c = B.h_ctls[i];
        ffmg_solve_info inf{};
        inf.cycles = std::max(c.k, 0);
        inf.vcycles = inf.cycles * B.inner;
        const double bn = sqrt(c.b2), rk = sqrt(c.rk2), r0 = sqrt(c.r0_2);
        inf.rel_residual = bn > 0 ? rk / bn : 0.0;
        inf.conv_factor = (inf.cycles > 0 && r0 > 0) ? pow(rk / r0, 1.0 / inf.cycles) : 0.0;
        inf.t_solve_ms = ms;
        inf.status = (c.done == 1) ? FFMG_OK : (c.done == 4 && c.k == 0) ? FFMG_ENAN : FFMG_ENOCONV;
        if (inf.status != FFMG_OK && worst == FFMG_OK) worst = (ffmg_status)inf.status;
        kmax = std::max(kmax, inf.cycles);
        if (infos) infos[i] = inf;
    }
    B.last_steps = kmax;
    if (worst != FFMG_OK) return fail(h0, worst, "some instances did not converge");
    return FFMG_OK;
}

ffmg_status farfield_map_batched(ffmg_handle *const *hs, int count, const double *etas, void *const *u, int n_dirs,
                                 const double *dirs, void *F)
{
    if (!hs || count < 1 || !hs[0]) return FFMG_EINVAL;
    ffmg_handle *h0 = hs[0];
    if (!etas || !F || !dirs || n_dirs < 1) return fail(h0, FFMG_EINVAL, "null argument or n_dirs < 1");
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, F) == hipSuccess)
        on_device = (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
    else
        (void)hipGetLastError();
    cd *Fd = (cd *)F;
    const size_t tot = (size_t)count * n_dirs;
    if (!on_device) {
        if (h0->d_F_cap < (int)tot) {
            TRY(dalloc(h0, &h0->d_F, tot * sizeof(cd)));
            h0->d_F_cap = (int)tot;
        }
        Fd = h0->d_F;
    }
    // 2D split-BF16 maps: every instance's stages in shared launches on
    // hs[0]'s stream, once each operator's plan is prepared for the directions
    bool batched = true;
    for (int i = 0; i < count && batched; ++i) {
        ffmg_handle *h = hs[i];
        if (!h) return fail(h0, FFMG_EINVAL, "hs[%d] is null", i);
        batched = h->prob.dim == 2 && h->opt.ff_precision == h0->opt.ff_precision &&
                  h->opt.ff_precision != FFMG_FF_FP64 && !h->pend.active;
    }
    if (batched) {
        std::vector<FFBInst> in(count);
        std::vector<uint64_t> key;
        std::vector<ffmg_handle *> seen;
        for (int i = 0; i < count; ++i) {
            ffmg_handle *h = hs[i];
            if (std::find(seen.begin(), seen.end(), h) == seen.end()) {
                TRY(farfield_prepare(h, etas + 3 * i, n_dirs, dirs));
                seen.push_back(h);
            }
            const LevelGeom &g = h->L[0].g;
            in[i] = FFBInst{h->ff, &g, h->L[0].q, u ? (const cd *)u[i] : nullptr, Fd + (size_t)i * n_dirs,
                            {etas[3 * i], etas[3 * i + 1], 0.0}, h->k0, h->prob.gamma};
            key.push_back(h->serial);
        }
        // the workspace keeps pointers into each plan (factor planes, direction
        // order): it is rebuilt when a plan was, or a tile variant changed
        for (ffmg_handle *h : seen) {
            key.push_back(ff_plan_generation(h->ff));
            key.push_back((uint64_t)ff_plan_variant(h->ff));
        }
        key.push_back((uint64_t)n_dirs);
        for (ffmg_handle *h : seen)
            if (h->stream != h0->stream) HIPCHK(h0, hipStreamSynchronize(h->stream));
        HIPCHK(h0, ff_batch_run(&h0->ffbatch, key, in, n_dirs, h0->stream));
        if (!on_device) HIPCHK(h0, hipMemcpyAsync(F, Fd, tot * sizeof(cd), hipMemcpyDeviceToHost, h0->stream));
        HIPCHK(h0, hipStreamSynchronize(h0->stream));
        return FFMG_OK;
    }
    std::vector<hipStream_t> streams;
    for (int i = 0; i < count; ++i) {
        ffmg_handle *h = hs[i];
        TRY(farfield_enqueue(h, etas + 3 * i, u ? u[i] : nullptr, n_dirs, dirs, Fd + (size_t)i * n_dirs));
        if (std::find(streams.begin(), streams.end(), h->stream) == streams.end()) streams.push_back(h->stream);
        if (h != h0 && h->err.size()) h0->err = h->err;
    }
    if (!on_device) {
        for (hipStream_t s : streams)
            if (s != h0->stream) HIPCHK(h0, hipStreamSynchronize(s));
        HIPCHK(h0, hipMemcpyAsync(F, Fd, tot * sizeof(cd), hipMemcpyDeviceToHost, h0->stream));
    }
    for (hipStream_t s : streams) HIPCHK(h0, hipStreamSynchronize(s));
    HIPCHK(h0, hipStreamSynchronize(h0->stream));
    return FFMG_OK;
}

}  // extern "C"
