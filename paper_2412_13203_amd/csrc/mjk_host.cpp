// mjk_host.cpp -- the C ABI of include/mjk.h: validation, the host planner
// and the launch sequence.
//
// Planner (Section 5, the two stages of building compute blocks):
//   stage 1: every shell pair A >= B is formed once, oriented l(A) >= l(B);
//            its primitive pairs go to a device table (k_pair_table) and its
//            Schwarz factor Q_AB = sqrt(max (ab|ab)) is computed on the device;
//            pairs are then sorted by angular-momentum class and primitive
//            count (bins), and by Q descending inside a bin;
//   stage 2: a bin pair (X, Y) forms the quartet blocks of one class; for each
//            bra pair of X the kept kets of Y are a prefix of Y (Q-sorted,
//            Q_AB Q_CD >= tau), cut into chunks of 64 q kets (q quartets per
//            lane, per class: the tile table of Algorithm 2), one wave each.
// Quartets themselves are never stored: only per-bra prefix lengths.
// Launches: one per (quartet class, precision); its segments are the bin
// pairs of that class, of one molecule (plan) or of many (batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mjk.h"
// generated class table (an ablation build names its own generated directory)
#ifndef MJK_GEN_DISPATCH
#define MJK_GEN_DISPATCH "gen/dispatch.inc"
#endif
#include MJK_GEN_DISPATCH
#include "mjk_types.hpp"
#include "stage_guard.hpp"

namespace mjk {
int launch_pair_table(const ShellPairD *pairs, int npair, const double *xyz, const int32_t *atom,
                      const int32_t *prim_off, const int32_t *nprim, const double *exps, const double *coefs,
                      PrimPairD *out, int nprim_pair, hipStream_t s);
int launch_fill(double *x, int64_t n, double v, hipStream_t s);
int launch_symmetrize(double *M, int n, hipStream_t s);
int launch_e2(const double *D, const double *J, const double *K, int n, double *e2, hipStream_t s);
int launch_fill_u32(uint32_t *x, int64_t n, uint32_t v, hipStream_t s);
int launch_stamp_init(unsigned long long *x, int n, hipStream_t s);
int launch_e2_grad_D(const double *J, const double *K, const double *g, double *out, int64_t n, hipStream_t s);
int launch_scale(double *x, int64_t n, const double *g, hipStream_t s);
int launch_boys(int mmax, const double *T, int64_t n, double *F, hipStream_t s);
int launch_rowmax_abs(const double *M, int n, double *out, hipStream_t s);
int launch_one_electron(const ShellPairD *pairs, const PrimPairD *prims, const int32_t *cls_idx,
                        const int32_t *cls_off, int lmax, const double *xyz, const double *Z, int natom, int nbf,
                        double *S, double *T, double *V, double *enuc, hipStream_t s);
int boys_lmax();
}  // namespace mjk

using namespace mjk;

struct mjk_ctx {
    int device;
    std::string arch;
    int ncu;
    std::mutex err_mu;  // last failure of a call made with this context
    std::string err;
    char *scratch = nullptr;  // this device's copy of the static scratch (device address)
};

namespace {

// Scratch of mjk_build_jk_static, for callers that cannot allocate device
// memory: the persistent kernels' work counters (first kStaticQueueBytes)
// and the split classes' staging slots (the rest).  Each device the library
// runs on holds its own copy for the life of the process; in host code the
// name only stands for the symbol, so its device address is looked up once
// per device (static_scratch_ptr) and only that address is used.
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
constexpr size_t kStaticQueueBytes = 4096;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
char *g_scratch_ptr[256];  // per device ordinal, filled on first use

}  // namespace

namespace {

thread_local std::string g_err;
thread_local mjk_ctx *g_cur_ctx = nullptr;  // context of the call running on this thread

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    if (g_cur_ctx) {
        std::lock_guard<std::mutex> lk(g_cur_ctx->err_mu);
        g_cur_ctx->err = buf;
    }
    return code;
}

// Marks the context of an entry point for its duration, so that a failure
// is recorded on that context as well as on the calling thread.
struct CtxScope {
    mjk_ctx *prev;
    explicit CtxScope(mjk_ctx *c) : prev(g_cur_ctx) { g_cur_ctx = c; }
    ~CtxScope() { g_cur_ctx = prev; }
};

#define HIP_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(MJK_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

inline int pair_class(int la, int lb) { return la * (la + 1) / 2 + lb; }
inline int quartet_class(int X, int Y) { return X * (X + 1) / 2 + Y; }
inline int ncart_h(int l) { return (l + 1) * (l + 2) / 2; }

// K-buckets of the primitive-pair count K_A K_B (waves stay uniform in it)
inline int kbucket(int np)
{
    if (np <= 1) return 0;
    if (np <= 4) return 1;
    if (np <= 9) return 2;
    if (np <= 16) return 3;
    if (np <= 25) return 4;
    return 5;
}
constexpr int kNumKBuckets = 6;
constexpr int kChunk = 64;          // kets per work item and quartet per lane
constexpr int kMaxQpl = 16;         // largest quartets-per-lane setting
constexpr int kEriStage = 65536;    // eri_class items per upload
constexpr int kEriSlots = 8;        // staging slots for eri_class / Schwarz without the plan's own
constexpr int kEriDeconstructMax = 4096;  // eri_class: split-class groups up to this size run one quartet per block
constexpr int kSlotsPerCU = 8;      // resident waves per CU the staging is sized for
constexpr int kGradMaxAtoms = 1024; // gradient: per-block copy of the gradient in LDS

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Bin {
    int cls, kb;
    int begin, count;  // positions in the sorted pair order
    int nrun;          // distinct first shells (runs) among its pairs
};

struct BinPair {
    int X, Y;          // bin indices, X >= Y in (class, bucket) order
    int qcls;          // quartet class index
};

// One segment: the FP64 or the FP32 part of one bin pair's quartets.
struct WorkList {
    int bp;            // bin pair
    int fp32;          // 1: FP32 recurrence (Q_AB Q_CD < fp32_tau)
    size_t off;        // int offset in the work-list region:
                       //   ket_count[nbra], run_begin[nbra + 1], chunk_prefix[nbra + 1]
    int nbra;
    int chunk;         // kets per item
    int nitems;
    int64_t nq;        // kept quartets
    int64_t npq;       // kept primitive quartets
    double cost;       // algorithmic flops
    double gcost;      // algorithmic flops of the gradient
};

// flops per primitive quartet outside the vertical recurrence: geometry (26),
// Boys (Taylor 4(K-1) + 2, downward 3L) and prefactor scaling (L+1)
inline double prim_overhead_flops(int L) { return 26.0 + 4.0 * 7 + 2.0 + 3.0 * L + (L + 1); }

}  // namespace

namespace {

// One launch: the segments of one quartet class at one precision.
struct Group {
    int qcls = 0, fp32 = 0;
    std::vector<std::pair<int, int>> segs;  // (molecule, work list), costliest per item first
    size_t seg_begin = 0;                   // first JKSeg of this launch in the segment array
    int nitems = 0;
    int64_t nq = 0, npq = 0;
    double cost = 0.0, gcost = 0.0;
};

}  // namespace

struct mjk_plan {
    mjk_ctx *ctx;
    // host copy of the basis
    int natom = 0, nshell = 0, nbf = 0;
    int64_t nprim = 0;
    std::vector<double> xyz, exps, coefs;
    std::vector<int32_t> atom, l, np, poff, ao;
    mjk_jk_opts opts{};
    // pairs
    int npair = 0;
    int64_t nprim_pair = 0;
    std::vector<ShellPairD> pairs_nat;   // natural order A(A+1)/2 + B
    std::vector<double> Q;               // natural order
    std::vector<int32_t> sorted;         // sorted position -> natural index
    std::vector<Bin> bins;
    std::vector<BinPair> bps;
    std::vector<WorkList> lists;         // bin pair x precision, natural order
    std::vector<int32_t> work;           // host copy of the work-list region
    std::vector<std::vector<int32_t>> class_pairs;  // natural indices per pair class
    std::vector<int32_t> class_off;      // pair class c: device list entries [class_off[c], class_off[c+1])
    int qpl[kNumQuartetClasses * kNumKBuckets];  // quartets per lane, per (class, bra K-bucket)
    std::vector<Group> groups;
    // class-sorted pair table (host copy) and the runs of every bin: bin-relative start, length
    std::vector<ShellPairD> psort;
    std::vector<std::vector<std::pair<int, int>>> bin_runs;
    bool dens_screen = false;            // work lists carry a density-weighted screen
    // staging lent by a batch while it binds its molecules (Schwarz factors of split classes)
    double *lent_stage = nullptr;
    size_t lent_stage_bytes = 0;
    int lent_nslot = 0;
    // workspace layout (byte offsets)
    size_t o_xyz, o_atom, o_poff, o_np, o_exps, o_coefs, o_pnat, o_psort, o_prims, o_Q, o_cls, o_work, o_runs,
        o_segs, o_queue, o_eri, o_rowmax, o_stage, o_stage_eri, total;
    size_t max_runs = 0;      // kept-run records: bound over all screening outcomes
    int nslot = 0;            // staging slots for split classes (0 with MJK_FLAG_NO_STAGING)
    int nslot_max = 0;        // slots a launch of this plan can use (occupancy bound)
    size_t stage_nacc = 0;    // largest split-class accumulator count present (J/K and gradient)
    int64_t max_items = 0;    // upper bound of the items of one segment (one quartet per lane)
    size_t work_ints = 0;
    bool in_batch = false;    // staging and launches belong to a batch
    size_t stage_bytes() const { return sizeof(double) * 64 * stage_nacc * (size_t)nslot; }
    char *ws = nullptr;
    bool bound = false;
    mjk_plan_stats stats{};
    // optional per-launch timing
    bool timing = false, timed_last = false, timed_grad = false;
    std::vector<hipEvent_t> ev;  // 2 per launch
    ~mjk_plan()
    {
        for (auto e : ev) hipEventDestroy(e);
    }
};

struct mjk_batch {
    mjk_ctx *ctx;
    std::vector<mjk_plan *> plans;
    std::vector<size_t> ws_off;      // each molecule's plan workspace inside the batch workspace
    std::vector<int64_t> mat_off;    // nmol + 1: packed D, J, K element offsets
    size_t o_segs = 0, o_queue = 0, o_stamps = 0, o_stage = 0, total = 0;
    size_t nseg = 0;
    int nslot = 0;
    size_t stage_nacc = 0;
    int qpl[kNumQuartetClasses * kNumKBuckets];
    std::vector<Group> groups;
    char *ws = nullptr;
    bool bound = false;
    bool stamps = false, stamped_last = false;
    size_t stage_bytes() const { return sizeof(double) * 64 * stage_nacc * (size_t)nslot; }
    bool timing = false, timed_last = false;
    std::vector<hipEvent_t> ev;
    ~mjk_batch()
    {
        for (auto e : ev) hipEventDestroy(e);
        for (auto *p : plans) delete p;
    }
};

namespace {

// Staging slots that eri_class and the Schwarz factors of split classes use:
// the plan's own (J/K) slots, or its small eri region.
struct StageView {
    double *ptr;
    size_t bytes;
    int nslot;
};

StageView eri_stage(const mjk_plan *p)
{
    if (p->nslot > 0) return {(double *)(p->ws + p->o_stage), p->stage_bytes(), p->nslot};
    if (p->lent_nslot > 0) return {p->lent_stage, p->lent_stage_bytes, p->lent_nslot};
    const size_t slot = sizeof(double) * 64 * p->stage_nacc;
    return {(double *)(p->ws + p->o_stage_eri), slot * kEriSlots, slot ? kEriSlots : 0};
}

// Classes with an f shell run in FP64 whatever fp32_tau is.
inline bool fp32_allowed(const ClassEntry &ce) { return std::max(std::max(ce.la, ce.lb), std::max(ce.lc, ce.ld)) < 3; }

// chunk prefix and item count of every work list of class `qcls` (-1: all)
// for the plan's quartets-per-lane table
void rechunk(mjk_plan *p, int qcls)
{
    for (auto &wl : p->lists) {
        const int qc = p->bps[wl.bp].qcls;
        if (qcls >= 0 && qc != qcls) continue;
        wl.chunk = kChunk * p->qpl[qc * kNumKBuckets + p->bins[p->bps[wl.bp].X].kb];
        const int32_t *cnt = p->work.data() + wl.off;
        int32_t *pre = p->work.data() + wl.off + 2 * (size_t)wl.nbra + 1;
        pre[0] = 0;
        for (int b = 0; b < wl.nbra; ++b) pre[b + 1] = pre[b] + (cnt[b] + wl.chunk - 1) / wl.chunk;
        wl.nitems = pre[wl.nbra];
    }
}

JKSeg make_seg(const mjk_plan *p, const WorkList &wl, int64_t mat_off, int mol)
{
    const BinPair &bp = p->bps[wl.bp];
    const Bin &X = p->bins[bp.X], &Y = p->bins[bp.Y];
    const char *w = p->ws;
    const int32_t *wk = (const int32_t *)(w + p->o_work) + wl.off;
    JKSeg g{};
    g.pairs = (const ShellPairD *)(w + p->o_psort);
    g.prims = (const PrimPairD *)(w + p->o_prims);
    g.runs = (const KetRun *)(w + p->o_runs);
    g.ket_count = wk;
    g.run_begin = wk + X.count;
    g.chunk_prefix = wk + 2 * X.count + 1;
    g.shell_atom = (const int32_t *)(w + p->o_atom);
    g.mat_off = mat_off;
    g.nbf = p->nbf;
    g.bra_begin = X.begin;
    g.nbra = X.count;
    g.ket_begin = Y.begin;
    g.same_bin = bp.X == bp.Y;
    g.chunk = wl.chunk;
    g.item_begin = 0;
    g.mol = mol;
    g.grad_off = 0;
    g.natom = p->natom;
    return g;
}

// Launch groups over the molecules' work lists: one per (class, precision),
// segments costliest per item first (longest-first inside the launch),
// launches costliest first.
std::vector<Group> make_groups(const std::vector<mjk_plan *> &plans)
{
    std::vector<Group> gs(2 * kNumQuartetClasses);
    for (int q = 0; q < kNumQuartetClasses; ++q)
        for (int f = 0; f < 2; ++f) {
            gs[2 * q + f].qcls = q;
            gs[2 * q + f].fp32 = f;
        }
    for (int m = 0; m < (int)plans.size(); ++m) {
        const mjk_plan *p = plans[m];
        for (int li = 0; li < (int)p->lists.size(); ++li) {
            const WorkList &wl = p->lists[li];
            if (wl.nitems <= 0) continue;
            Group &g = gs[2 * p->bps[wl.bp].qcls + wl.fp32];
            g.segs.push_back({m, li});
            g.nitems += wl.nitems;
            g.nq += wl.nq;
            g.npq += wl.npq;
            g.cost += wl.cost;
            g.gcost += wl.gcost;
        }
    }
    std::vector<Group> out;
    for (auto &g : gs) {
        if (g.nitems == 0) continue;
        std::stable_sort(g.segs.begin(), g.segs.end(), [&](const std::pair<int, int> &x, const std::pair<int, int> &y) {
            const WorkList &a = plans[x.first]->lists[x.second], &b = plans[y.first]->lists[y.second];
            return a.cost / a.nitems > b.cost / b.nitems;
        });
        out.push_back(std::move(g));
    }
    std::stable_sort(out.begin(), out.end(), [](const Group &a, const Group &b) { return a.cost > b.cost; });
    size_t off = 0;
    for (auto &g : out) {
        g.seg_begin = off;
        off += g.segs.size();
    }
    return out;
}

// segment records of every group, uploaded to dsegs (synchronous on s)
int upload_groups(const std::vector<Group> &gs, const std::vector<mjk_plan *> &plans, const int64_t *mat_off,
                  JKSeg *dsegs, hipStream_t s)
{
    std::vector<JKSeg> h;
    for (const auto &g : gs) {
        int item = 0;
        for (const auto &sm : g.segs) {
            const mjk_plan *p = plans[sm.first];
            JKSeg seg = make_seg(p, p->lists[sm.second], mat_off[sm.first], sm.first);
            seg.item_begin = item;
            item += p->lists[sm.second].nitems;
            h.push_back(seg);
        }
    }
    if (h.empty()) return MJK_OK;
    HIP_TRY(hipMemcpyAsync(dsegs, h.data(), sizeof(JKSeg) * h.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // h is released on return
    return MJK_OK;
}

int upload_work(mjk_plan *p, hipStream_t s)
{
    if (p->work.empty()) return MJK_OK;
    HIP_TRY(hipMemcpyAsync(p->ws + p->o_work, p->work.data(), sizeof(int32_t) * p->work.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MJK_OK;
}

int ensure_events(std::vector<hipEvent_t> &ev, size_t n)
{
    if (ev.size() == n) return MJK_OK;
    for (auto e : ev) hipEventDestroy(e);
    ev.assign(n, nullptr);
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    return MJK_OK;
}

// Run every group: J/K (grad == nullptr) or the gradient.  The caller has
// cleared the outputs; the work counters are cleared here.
int run_groups(const std::vector<Group> &gs, const JKSeg *dsegs, uint32_t *dqueue, double *stage, size_t stage_bytes,
               int nslot, const double *D, double *J, double *K, double *grad, int natom_max,
               unsigned long long *stamps, hipStream_t s, std::vector<hipEvent_t> *ev, const char *who,
               bool lane_persistent = false)
{
    if (gs.empty()) return MJK_OK;
    if (launch_fill_u32(dqueue, (int64_t)gs.size(), 0u, s)) return fail(MJK_ERR_HIP, "%s: fill launch failed", who);
    for (size_t i = 0; i < gs.size(); ++i) {
        const Group &g = gs[i];
        JKLaunch a{};
        a.segs = dsegs + g.seg_begin;
        a.nseg = (int32_t)g.segs.size();
        a.nitems = g.nitems;
        a.D = D;
        a.J = J;
        a.K = K;
        a.grad = grad;
        a.stage = stage;
        a.stage_bytes = stage_bytes;
        a.nslot = nslot;
        a.natom_max = natom_max;
        a.queue = dqueue + i;
        a.stamps = stamps;
        a.lane_persistent = lane_persistent ? 1 : 0;
        const ClassEntry &ce = kClassTable[g.qcls];
        if (ev) HIP_TRY(hipEventRecord((*ev)[2 * i], s));
        if (grad && !ce.grad) return fail(MJK_ERR_UNSUPPORTED, "%s: no gradient kernel for this class", who);
        const int rc = grad ? ce.grad(a, s) : (g.fp32 ? ce.jk32(a, s) : ce.jk(a, s));
        if (rc == kLaunchStaging)
            return fail(MJK_ERR_STATE, "%s: class (%d%d|%d%d): the staging region (%zu bytes, %d slots) cannot hold "
                        "one slot per block of the launch", who, ce.la, ce.lb, ce.lc, ce.ld, stage_bytes, nslot);
        if (rc) return fail(MJK_ERR_HIP, "%s: class launch failed", who);
        if (ev) HIP_TRY(hipEventRecord((*ev)[2 * i + 1], s));
    }
    return MJK_OK;
}

int fill_timings(const std::vector<Group> &gs, std::vector<hipEvent_t> &ev, bool grad, mjk_class_timing *out,
                 int32_t cap, int32_t *n)
{
    std::vector<mjk_class_timing> acc(kNumQuartetClasses);
    for (int q = 0; q < kNumQuartetClasses; ++q) {
        acc[q] = mjk_class_timing{};
        acc[q].la = kClassTable[q].la;
        acc[q].lb = kClassTable[q].lb;
        acc[q].lc = kClassTable[q].lc;
        acc[q].ld = kClassTable[q].ld;
    }
    for (size_t i = 0; i < gs.size(); ++i) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
        auto &t = acc[gs[i].qcls];
        t.nlaunch += 1;
        t.ms += ms;
        t.nquartet += gs[i].nq;
        t.nprim_quartet += gs[i].npq;
        t.flops += grad ? gs[i].gcost : gs[i].cost;
    }
    int k = 0;
    for (int q = 0; q < kNumQuartetClasses; ++q)
        if (acc[q].nlaunch > 0) {
            if (k < cap) out[k] = acc[q];
            ++k;
        }
    *n = k;
    return MJK_OK;
}

constexpr int kTileUnits = kNumQuartetClasses * kNumKBuckets;

// Validates a tile table of n = classes (one value per class) or n = classes
// x K-buckets (one per class and bra K-bucket) entries and expands it into
// the per-unit table `units`.
int check_qpl(const int32_t *qpl, int32_t n, const char *who, int *units)
{
    if (!qpl || (n != kNumQuartetClasses && n != kTileUnits))
        return fail(MJK_ERR_INVALID_ARG, "%s: need %d per-class or %d per-class-and-bucket values", who,
                    kNumQuartetClasses, kTileUnits);
    for (int q = 0; q < n; ++q) {
        const int v = qpl[q];
        if (v < 1 || v > kMaxQpl || (v & (v - 1)))
            return fail(MJK_ERR_INVALID_ARG, "%s: entry %d: %d quartets per lane (1, 2, 4, ... %d)", who, q, v,
                        kMaxQpl);
    }
    for (int u = 0; u < kTileUnits; ++u) units[u] = n == kTileUnits ? qpl[u] : qpl[u / kNumKBuckets];
    return MJK_OK;
}

}  // namespace

extern "C" {

int mjk_lmax(void) { return kLmax; }

int mjk_grad_lmax(void) { return kGradLmax; }

int mjk_num_classes(void) { return kNumQuartetClasses; }

int mjk_class_l(int32_t q, int32_t *l4)
{
    if (q < 0 || q >= kNumQuartetClasses || !l4) return fail(MJK_ERR_INVALID_ARG, "mjk_class_l: bad argument");
    l4[0] = kClassTable[q].la;
    l4[1] = kClassTable[q].lb;
    l4[2] = kClassTable[q].lc;
    l4[3] = kClassTable[q].ld;
    return MJK_OK;
}

const char *mjk_last_error(void) { return g_err.c_str(); }

const char *mjk_ctx_last_error(mjk_ctx *ctx)
{
    if (!ctx) return "";
    thread_local std::string copy;
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    copy = ctx->err;
    return copy.c_str();
}

int mjk_boys(mjk_ctx *ctx, int32_t mmax, const double *T, int64_t n, double *F, void *stream)
{
    if (!ctx) return fail(MJK_ERR_INVALID_ARG, "mjk_boys: ctx is NULL");
    CtxScope cs_(ctx);
    if (mmax < 0 || mmax > boys_lmax())
        return fail(MJK_ERR_UNSUPPORTED, "mjk_boys: mmax = %d outside 0..%d", mmax, boys_lmax());
    if (n < 0 || (n > 0 && (!T || !F))) return fail(MJK_ERR_INVALID_ARG, "mjk_boys: bad arguments");
    if (n == 0) return MJK_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    if (launch_boys(mmax, T, n, F, (hipStream_t)stream)) return fail(MJK_ERR_HIP, "mjk_boys: launch failed");
    return MJK_OK;
}

int mjk_ctx_create(int device, mjk_ctx **out)
{
    if (!out) return fail(MJK_ERR_INVALID_ARG, "mjk_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
        return fail(MJK_ERR_NO_DEVICE, "mjk_ctx_create: no HIP device");
    if (device < 0 || device >= n) return fail(MJK_ERR_NO_DEVICE, "mjk_ctx_create: device %d of %d", device, n);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0)
        return fail(MJK_ERR_NO_DEVICE, "mjk_ctx_create: device %d is %s, the library targets gfx950", device,
                    arch.c_str());
    char *scr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device >= 256) return fail(MJK_ERR_NO_DEVICE, "mjk_ctx_create: device ordinal %d too large", device);
        if (!g_scratch_ptr[device]) {
            // with the device current: its copy of the static scratch
            HIP_TRY(hipSetDevice(device));
            void *ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr || ((uintptr_t)ptr & 255) != 0)
                return fail(MJK_ERR_HIP, "mjk_ctx_create: static scratch address %p", ptr);
            g_scratch_ptr[device] = (char *)ptr;
        }
        scr = g_scratch_ptr[device];
    }
    auto *c = new mjk_ctx;
    c->device = device;
    c->arch = arch;
    c->ncu = prop.multiProcessorCount;
    c->scratch = scr;
    *out = c;
    return MJK_OK;
}

void mjk_ctx_destroy(mjk_ctx *ctx) { delete ctx; }

}  // extern "C"

static int validate_basis(const mjk_basis *b)
{
    if (!b) return fail(MJK_ERR_INVALID_ARG, "basis is NULL");
    if (b->natom <= 0 || b->nshell <= 0 || b->nprim <= 0)
        return fail(MJK_ERR_INVALID_ARG, "basis: natom=%d nshell=%d nprim=%lld must be positive", b->natom,
                    b->nshell, (long long)b->nprim);
    if (!b->xyz || !b->shell_atom || !b->shell_l || !b->shell_nprim || !b->shell_prim_off || !b->exps ||
        !b->coefs)
        return fail(MJK_ERR_INVALID_ARG, "basis: NULL array");
    for (int i = 0; i < 3 * b->natom; ++i)
        if (!std::isfinite(b->xyz[i])) return fail(MJK_ERR_INVALID_ARG, "basis: xyz[%d] is not finite", i);
    for (int s = 0; s < b->nshell; ++s) {
        const int l = b->shell_l[s], k = b->shell_nprim[s], o = b->shell_prim_off[s], a = b->shell_atom[s];
        if (l < 0) return fail(MJK_ERR_INVALID_ARG, "basis: shell %d has l=%d", s, l);
        if (l > kLmax) return fail(MJK_ERR_UNSUPPORTED, "basis: shell %d has l=%d > %d", s, l, kLmax);
        if (k < 1 || k > 6) return fail(MJK_ERR_UNSUPPORTED, "basis: shell %d has %d primitives (1..6)", s, k);
        if (a < 0 || a >= b->natom) return fail(MJK_ERR_INVALID_ARG, "basis: shell %d on atom %d", s, a);
        if (o < 0 || (int64_t)o + k > b->nprim)
            return fail(MJK_ERR_INVALID_ARG, "basis: shell %d primitives [%d, %d) outside [0, %lld)", s, o, o + k,
                        (long long)b->nprim);
        for (int i = 0; i < k; ++i) {
            const double e = b->exps[o + i], c = b->coefs[o + i];
            if (!(std::isfinite(e) && e > 0.0))
                return fail(MJK_ERR_INVALID_ARG, "basis: shell %d exponent %d = %g", s, i, e);
            if (!std::isfinite(c)) return fail(MJK_ERR_INVALID_ARG, "basis: shell %d coefficient %d = %g", s, i, c);
        }
    }
    return MJK_OK;
}

static int plan_create(mjk_ctx *ctx, const mjk_basis *b, const mjk_jk_opts *opts, bool in_batch, mjk_plan **out,
                       size_t *ws_bytes)
{
    if (!ctx || !out || !ws_bytes) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: NULL argument");
    CtxScope cs_(ctx);
    *out = nullptr;
    if (int rc = validate_basis(b)) return rc;
    mjk_jk_opts o{};
    if (opts) o = *opts;
    if (!(std::isfinite(o.schwarz_tau) && o.schwarz_tau >= 0.0))
        return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: schwarz_tau = %g", o.schwarz_tau);
    if (!(std::isfinite(o.fp32_tau) && o.fp32_tau >= 0.0))
        return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: fp32_tau = %g", o.fp32_tau);
    if (o.flags & ~(MJK_FLAG_CHECK | MJK_FLAG_GRAD | MJK_FLAG_NO_STAGING | MJK_FLAG_PERSISTENT | MJK_FLAG_NO_KBINS))
        return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: unknown flags 0x%x", o.flags);
    if ((o.flags & MJK_FLAG_NO_STAGING) && (in_batch || (o.flags & MJK_FLAG_GRAD)))
        return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: MJK_FLAG_NO_STAGING is for single J/K plans only");
    if (o.flags & MJK_FLAG_GRAD)
        for (int s = 0; s < b->nshell; ++s)
            if (b->shell_l[s] > kGradLmax)
                return fail(MJK_ERR_UNSUPPORTED, "mjk_plan_create: gradient plan: shell %d has l=%d > %d", s,
                            b->shell_l[s], kGradLmax);

    auto *p = new mjk_plan;
    p->ctx = ctx;
    p->opts = o;
    p->in_batch = in_batch;
    for (int q = 0; q < kNumQuartetClasses * kNumKBuckets; ++q) p->qpl[q] = 1;
    p->natom = b->natom;
    p->nshell = b->nshell;
    p->nprim = b->nprim;
    p->xyz.assign(b->xyz, b->xyz + 3 * b->natom);
    p->exps.assign(b->exps, b->exps + b->nprim);
    p->coefs.assign(b->coefs, b->coefs + b->nprim);
    p->atom.assign(b->shell_atom, b->shell_atom + b->nshell);
    p->l.assign(b->shell_l, b->shell_l + b->nshell);
    p->np.assign(b->shell_nprim, b->shell_nprim + b->nshell);
    p->poff.assign(b->shell_prim_off, b->shell_prim_off + b->nshell);
    p->ao.resize(b->nshell + 1);
    p->ao[0] = 0;
    for (int s = 0; s < b->nshell; ++s) p->ao[s + 1] = p->ao[s] + ncart_h(p->l[s]);
    p->nbf = p->ao[b->nshell];

    // stage 1 on the host side: the oriented pair list (natural order)
    const int ns = p->nshell;
    p->npair = ns * (ns + 1) / 2;
    p->pairs_nat.resize(p->npair);
    p->class_pairs.assign(kNumPairClasses, {});
    int64_t pp = 0;
    for (int A = 0, k = 0; A < ns; ++A)
        for (int B = 0; B <= A; ++B, ++k) {
            int s1 = A, s2 = B;
            if (p->l[s2] > p->l[s1]) std::swap(s1, s2);
            ShellPairD &sp = p->pairs_nat[k];
            sp.A = s1;
            sp.B = s2;
            sp.prim_off = (int32_t)pp;
            sp.nprim = p->np[s1] * p->np[s2];
            sp.ao_a = p->ao[s1];
            sp.ao_b = p->ao[s2];
            sp.same = (A == B);
            sp.cls = pair_class(p->l[s1], p->l[s2]);
            for (int x = 0; x < 3; ++x) sp.AB[x] = p->xyz[3 * p->atom[s1] + x] - p->xyz[3 * p->atom[s2] + x];
            sp.Q = 0.0;
            pp += sp.nprim;
            p->class_pairs[sp.cls].push_back(k);
        }
    p->nprim_pair = pp;
    if (pp > INT32_MAX) {
        delete p;
        return fail(MJK_ERR_UNSUPPORTED, "mjk_plan_create: %lld primitive pairs exceed int32", (long long)pp);
    }

    // bins by (class, K-bucket): sizes and runs (distinct first shells) known
    // now, the order inside a run (Q) decided at bind
    std::vector<int> bin_size(kNumPairClasses * kNumKBuckets, 0);
    std::vector<std::vector<int32_t>> bin_first(kNumPairClasses * kNumKBuckets);
    for (const auto &sp : p->pairs_nat) {
        const int key = sp.cls * kNumKBuckets + ((o.flags & MJK_FLAG_NO_KBINS) ? 0 : kbucket(sp.nprim));
        bin_size[key]++;
        bin_first[key].push_back(sp.A);
    }
    int pos = 0;
    for (int c = 0; c < kNumPairClasses; ++c)
        for (int kb = 0; kb < kNumKBuckets; ++kb) {
            const int key = c * kNumKBuckets + kb;
            const int n = bin_size[key];
            if (n == 0) continue;
            auto &f = bin_first[key];
            std::sort(f.begin(), f.end());
            const int nrun = (int)(std::unique(f.begin(), f.end()) - f.begin());
            p->bins.push_back({c, kb, pos, n, nrun});
            pos += n;
        }
    // bin pairs X >= Y (bin order = (class, bucket) order, so class(X) >= class(Y))
    size_t woff = 0;
    for (int X = 0; X < (int)p->bins.size(); ++X)
        for (int Y = 0; Y <= X; ++Y) {
            BinPair bp{};
            bp.X = X;
            bp.Y = Y;
            bp.qcls = quartet_class(p->bins[X].cls, p->bins[Y].cls);
            for (int prec = 0; prec < 2; ++prec) {
                WorkList wl{};
                wl.bp = (int)p->bps.size();
                wl.fp32 = prec;
                wl.off = woff;
                wl.nbra = p->bins[X].count;
                wl.chunk = kChunk;
                woff += 3 * (size_t)p->bins[X].count + 2;
                p->lists.push_back(wl);
                // a bra keeps at most one record per run of the ket bin; FP32
                // lists stay empty without an FP32 threshold
                if (prec == 0 || o.fp32_tau > 0.0) p->max_runs += (size_t)p->bins[X].count * p->bins[Y].nrun;
            }
            p->bps.push_back(bp);
        }
    p->work_ints = woff;
    if (p->max_runs > (size_t)INT32_MAX) {
        const size_t nr = p->max_runs;
        delete p;
        return fail(MJK_ERR_UNSUPPORTED, "mjk_plan_create: %zu kept-run records exceed int32", nr);
    }
    // split classes present: staging for one item per persistent block;
    // a launch never has more blocks than work items
    for (const auto &bp : p->bps) {
        const ClassEntry &ce = kClassTable[bp.qcls];
        size_t need = ce.split ? (size_t)ce.nacc : 0;
        if ((o.flags & MJK_FLAG_GRAD) && ce.grad_stage_nacc) need = std::max(need, ce.grad_stage_nacc());
        if (need == 0) continue;
        p->stage_nacc = std::max(p->stage_nacc, need);
        const int64_t ny = p->bins[bp.Y].count;
        p->max_items = std::max(p->max_items, (int64_t)p->bins[bp.X].count * ((ny + kChunk - 1) / kChunk));
    }
    p->nslot_max = p->stage_nacc ? (int)std::min<int64_t>(kSlotsPerCU * std::max(1, ctx->ncu), 2 * p->max_items) : 0;
    const bool own_staging = !in_batch && !(o.flags & MJK_FLAG_NO_STAGING);
    p->nslot = own_staging ? p->nslot_max : 0;

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o2 = off;
        off = align_up(off + bytes);
        return o2;
    };
    p->o_xyz = take(sizeof(double) * 3 * p->natom);
    p->o_atom = take(sizeof(int32_t) * ns);
    p->o_poff = take(sizeof(int32_t) * ns);
    p->o_np = take(sizeof(int32_t) * ns);
    p->o_exps = take(sizeof(double) * p->nprim);
    p->o_coefs = take(sizeof(double) * p->nprim);
    p->o_pnat = take(sizeof(ShellPairD) * p->npair);
    p->o_psort = take(sizeof(ShellPairD) * p->npair);
    p->o_prims = take(sizeof(PrimPairD) * (size_t)p->nprim_pair);
    p->o_Q = take(sizeof(double) * p->npair);
    p->o_cls = take(sizeof(int32_t) * p->npair);
    p->o_work = take(sizeof(int32_t) * p->work_ints);
    p->o_runs = take(sizeof(KetRun) * std::max<size_t>(p->max_runs, 1));
    p->o_segs = take(in_batch ? 0 : sizeof(JKSeg) * p->lists.size());
    p->o_queue = take(own_staging ? sizeof(uint32_t) * 2 * kNumQuartetClasses : 0);
    p->o_eri = take(sizeof(EriItem) * kEriStage);
    p->o_rowmax = take(sizeof(double) * p->nbf);
    p->o_stage = take(p->stage_bytes());
    // plans created with MJK_FLAG_NO_STAGING keep a few staging slots for
    // eri_class and the Schwarz factors of split classes (batch members
    // borrow the batch's staging while it binds them)
    p->o_stage_eri = take(p->nslot == 0 && !in_batch ? sizeof(double) * 64 * p->stage_nacc * kEriSlots : 0);
    p->total = off;

    p->stats.nbf = p->nbf;
    p->stats.nshell = ns;
    p->stats.npair = p->npair;
    p->stats.nprim_pair = p->nprim_pair;
    p->stats.nquartet_total = (int64_t)p->npair * (p->npair + 1) / 2;
    p->stats.workspace_bytes = p->total;
    *ws_bytes = p->total;
    *out = p;
    return MJK_OK;
}

// host threads for the planner's per-bin-pair loops: the hardware threads,
// capped by OMP_NUM_THREADS when set and at 16
static size_t host_threads()
{
    size_t n = std::max(1u, std::thread::hardware_concurrency());
    if (const char *e = std::getenv("OMP_NUM_THREADS")) {
        const long v = std::strtol(e, nullptr, 10);
        if (v > 0) n = std::min(n, (size_t)v);
    }
    return std::min<size_t>(n, 16);
}

// tables, Schwarz factors, sort and work lists of one plan (its workspace)
// Stage 2 of the plan: per bin pair, per bra, the kept prefix of every run of
// the ket bin as kept-run records, the work lists' chunking, the launch groups
// and their segments; uploads them (synchronizes s).  shell_w (host, one
// value per shell, or null): weights of a density-weighted screen with
// threshold tau_w, applied on top of the Schwarz screen.
static int build_lists(mjk_plan *p, const double *shell_w, double tau_w, hipStream_t s)
{
    // stage 2: per bin pair, per bra, the kept prefix of every run of the ket
    // bin (Q_AB Q_CD >= schwarz_tau; with coinciding bins also ket <= bra),
    // split into its FP64 part (Q_AB Q_CD >= fp32_tau) and FP32 remainder
    const double tau = p->opts.schwarz_tau, tau32 = p->opts.fp32_tau;
    const std::vector<ShellPairD> &psort = p->psort;
    const auto &bin_runs = p->bin_runs;
    char *w = p->ws;
    p->work.assign(p->work_ints, 0);
    std::vector<KetRun> runs;
    int64_t nq_kept = 0, nprimq = 0, ncart = 0, nq32 = 0;
    double flops = 0.0, gflops = 0.0;
    // kets of [lo, lo + n) (bin positions of Y, Q descending) with qb * Q >= thr
    auto kept_len = [&](const Bin &Y, int lo, int n, double qb, double thr) {
        int a0 = 0, a1 = n;
        while (a0 < a1) {
            const int mid = (a0 + a1) >> 1;
            if (qb * psort[Y.begin + lo + mid].Q < thr)
                a1 = mid;
            else
                a0 = mid + 1;
        }
        return a0;
    };
    // per run of every bin: max(w_C, max over its kets of w_D)
    std::vector<std::vector<double>> run_w;
    if (shell_w) {
        run_w.resize(p->bins.size());
        for (size_t y = 0; y < p->bins.size(); ++y) {
            const Bin &Y = p->bins[y];
            for (const auto &run : bin_runs[y]) {
                double m = shell_w[psort[Y.begin + run.first].A];
                for (int k = 0; k < run.second; ++k) m = std::max(m, shell_w[psort[Y.begin + run.first + k].B]);
                run_w[y].push_back(m);
            }
        }
    }
    // the bin pairs are independent: each fills its own counts and run
    // offsets (relative to its own records) on a host thread, then the
    // records are concatenated in list order, which fixes the layout
    struct ListRuns {
        std::vector<KetRun> r64, r32;
        int64_t q64 = 0, q32 = 0, pq64 = 0, pq32 = 0;
    };
    const size_t npl = p->lists.size() / 2;
    std::vector<ListRuns> lr(npl);
    auto fill_list = [&](size_t ip) {
        WorkList &l64 = p->lists[2 * ip], &l32 = p->lists[2 * ip + 1];
        const BinPair &bp = p->bps[l64.bp];
        const Bin &X = p->bins[bp.X], &Y = p->bins[bp.Y];
        const auto &yr = bin_runs[bp.Y];
        const ClassEntry &ce = kClassTable[bp.qcls];
        const double t32 = fp32_allowed(ce) ? tau32 : 0.0;
        int32_t *c64 = p->work.data() + l64.off, *rb64 = c64 + X.count;
        int32_t *c32 = p->work.data() + l32.off, *rb32 = c32 + X.count;
        std::vector<int64_t> ynp(Y.count + 1, 0);  // prefix of K_C K_D over the ket bin
        for (int k = 0; k < Y.count; ++k) ynp[k + 1] = ynp[k] + psort[Y.begin + k].nprim;
        ListRuns &o = lr[ip];
        for (int b = 0; b < X.count; ++b) {
            const double qb = psort[X.begin + b].Q;
            const int64_t nb = psort[X.begin + b].nprim;
            rb64[b] = (int32_t)o.r64.size();
            rb32[b] = (int32_t)o.r32.size();
            int n64 = 0, n32 = 0;
            const double wb = shell_w ? std::max(shell_w[psort[X.begin + b].A], shell_w[psort[X.begin + b].B]) : 0.0;
            for (size_t ri = 0; ri < yr.size(); ++ri) {
                const auto &run = yr[ri];
                int len = run.second;
                if (bp.X == bp.Y) {
                    if (run.first > b) break;
                    len = std::min(len, b - run.first + 1);
                }
                int keep = kept_len(Y, run.first, len, qb, tau);
                // density-weighted screen: Q_AB Q_CD max(w_A, w_B, w_C, max_D w_D) >= tau_w
                if (shell_w) keep = kept_len(Y, run.first, keep, qb * std::max(wb, run_w[bp.Y][ri]), tau_w);
                const int k64 = t32 > 0.0 ? std::min(keep, kept_len(Y, run.first, keep, qb, t32)) : keep;
                if (k64 > 0) {
                    o.r64.push_back({n64, run.first});
                    n64 += k64;
                    o.pq64 += nb * (ynp[run.first + k64] - ynp[run.first]);
                }
                if (keep > k64) {
                    o.r32.push_back({n32, run.first + k64});
                    n32 += keep - k64;
                    o.pq32 += nb * (ynp[run.first + keep] - ynp[run.first + k64]);
                }
            }
            c64[b] = n64;
            c32[b] = n32;
            o.q64 += n64;
            o.q32 += n32;
        }
        rb64[X.count] = (int32_t)o.r64.size();
        rb32[X.count] = (int32_t)o.r32.size();
    };
    {
        std::atomic<size_t> next{0};
        std::atomic<bool> failed{false};
        auto worker = [&]() {
            try {
                for (size_t ip; (ip = next.fetch_add(1)) < npl && !failed.load();) fill_list(ip);
            } catch (...) {
                failed = true;
            }
        };
        const int nth = (int)std::min<size_t>(host_threads(), std::max<size_t>(npl, 1));
        std::vector<std::thread> pool;
        try {
            for (int t = 1; t < nth; ++t) pool.emplace_back(worker);
        } catch (...) {  // fewer threads: the others take the remaining lists
        }
        worker();
        for (auto &t : pool) t.join();
        if (failed) return fail(MJK_ERR_UNSUPPORTED, "mjk_plan_bind: host memory exhausted by the kept-run records");
    }
    size_t nruns = 0;
    for (const auto &o : lr) nruns += o.r64.size() + o.r32.size();
    if (nruns > p->max_runs) return fail(MJK_ERR_STATE, "mjk_plan_bind: kept-run records exceed their bound");
    runs.reserve(nruns);
    for (size_t il = 0; il < p->lists.size(); il += 2) {
        WorkList &l64 = p->lists[il], &l32 = p->lists[il + 1];
        const BinPair &bp = p->bps[l64.bp];
        const Bin &X = p->bins[bp.X];
        const ClassEntry &ce = kClassTable[bp.qcls];
        int32_t *rb64 = p->work.data() + l64.off + X.count, *rb32 = p->work.data() + l32.off + X.count;
        ListRuns &o = lr[il / 2];
        const int32_t base64 = (int32_t)runs.size(), base32 = (int32_t)(runs.size() + o.r64.size());
        for (int b = 0; b <= X.count; ++b) {
            rb64[b] += base64;
            rb32[b] += base32;
        }
        runs.insert(runs.end(), o.r64.begin(), o.r64.end());
        runs.insert(runs.end(), o.r32.begin(), o.r32.end());
        std::vector<KetRun>().swap(o.r64);
        std::vector<KetRun>().swap(o.r32);
        const int64_t q64 = o.q64, q32 = o.q32, pq64 = o.pq64, pq32 = o.pq32;
        const int nout = ncart_h(ce.la) * ncart_h(ce.lb) * ncart_h(ce.lc) * ncart_h(ce.ld);
        const int L = ce.la + ce.lb + ce.lc + ce.ld;
        const double fpq = ce.vrr_flops + prim_overhead_flops(L), fq = ce.hrr_flops + 12.0 * nout;
        const double gpq = ce.grad_vrr_flops + ce.grad_nup * prim_overhead_flops(L + 1) +
                           ce.grad_ndown * (prim_overhead_flops(L - 1) + 1.0);
        l64.nq = q64;
        l64.npq = pq64;
        l64.cost = (double)pq64 * fpq + (double)q64 * fq;
        l64.gcost = (double)pq64 * gpq + (double)q64 * ce.grad_q_flops;
        l32.nq = q32;
        l32.npq = pq32;
        l32.cost = (double)pq32 * fpq + (double)q32 * fq;
        l32.gcost = (double)pq32 * gpq + (double)q32 * ce.grad_q_flops;
        nq_kept += q64 + q32;
        nq32 += q32;
        nprimq += pq64 + pq32;
        ncart += (q64 + q32) * nout;
        flops += l64.cost + l32.cost;
        gflops += l64.gcost + l32.gcost;
    }
    if (!runs.empty())
        HIP_TRY(hipMemcpyAsync(w + p->o_runs, runs.data(), sizeof(KetRun) * runs.size(), hipMemcpyHostToDevice, s));
    rechunk(p, -1);
    if (int rc = upload_work(p, s)) return rc;  // synchronizes: psort and runs are released on return
    p->stats.nquartet_kept = nq_kept;
    p->stats.nquartet_fp32 = nq32;
    p->stats.nprim_quartet_kept = nprimq;
    p->stats.ncart_eri_kept = ncart;
    p->stats.vrr_flops_kept = flops;
    p->stats.grad_flops_kept = (p->opts.flags & MJK_FLAG_GRAD) ? gflops : 0.0;
    if (!p->in_batch) {
        p->groups = make_groups({p});
        const int64_t zero = 0;
        if (int rc = upload_groups(p->groups, {p}, &zero, (JKSeg *)(w + p->o_segs), s)) return rc;
        p->stats.nlaunch = (int64_t)p->groups.size() + 4;
    }
    return MJK_OK;
}

static int plan_bind(mjk_plan *p, void *workspace, size_t bytes, hipStream_t s)
{
    if (!workspace) return fail(MJK_ERR_WORKSPACE, "mjk_plan_bind: workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(MJK_ERR_WORKSPACE, "mjk_plan_bind: workspace not 256-byte aligned");
    if (bytes < p->total)
        return fail(MJK_ERR_WORKSPACE, "mjk_plan_bind: workspace %zu bytes < %zu needed", bytes, p->total);
    HIP_TRY(hipSetDevice(p->ctx->device));
    p->ws = (char *)workspace;
    p->bound = false;
    char *w = p->ws;
    const int ns = p->nshell;
    HIP_TRY(hipMemcpyAsync(w + p->o_xyz, p->xyz.data(), sizeof(double) * 3 * p->natom, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + p->o_atom, p->atom.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + p->o_poff, p->poff.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + p->o_np, p->np.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + p->o_exps, p->exps.data(), sizeof(double) * p->nprim, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + p->o_coefs, p->coefs.data(), sizeof(double) * p->nprim, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w + p->o_pnat, p->pairs_nat.data(), sizeof(ShellPairD) * p->npair, hipMemcpyHostToDevice,
                           s));
    auto *pnat = (const ShellPairD *)(w + p->o_pnat);
    auto *prims = (PrimPairD *)(w + p->o_prims);
    auto *dQ = (double *)(w + p->o_Q);
    if (launch_pair_table(pnat, p->npair, (const double *)(w + p->o_xyz), (const int32_t *)(w + p->o_atom),
                          (const int32_t *)(w + p->o_poff), (const int32_t *)(w + p->o_np),
                          (const double *)(w + p->o_exps), (const double *)(w + p->o_coefs), prims,
                          (int)p->nprim_pair, s))
        return fail(MJK_ERR_HIP, "mjk_plan_bind: pair-table launch failed");
    // Schwarz factors per pair class
    std::vector<int32_t> cls_idx;
    std::vector<size_t> cls_off(kNumPairClasses + 1, 0);
    for (int c = 0; c < kNumPairClasses; ++c) {
        cls_off[c] = cls_idx.size();
        cls_idx.insert(cls_idx.end(), p->class_pairs[c].begin(), p->class_pairs[c].end());
    }
    cls_off[kNumPairClasses] = cls_idx.size();
    p->class_off.assign(cls_off.begin(), cls_off.end());
    auto *didx = (int32_t *)(w + p->o_cls);
    HIP_TRY(hipMemcpyAsync(didx, cls_idx.data(), sizeof(int32_t) * cls_idx.size(), hipMemcpyHostToDevice, s));
    for (int q = 0; q < kNumQuartetClasses; ++q) {
        const ClassEntry &ce = kClassTable[q];
        if (ce.la != ce.lc || ce.lb != ce.ld) continue;
        const int c = pair_class(ce.la, ce.lb);
        const int n = (int)(cls_off[c + 1] - cls_off[c]);
        if (n == 0) continue;
        if (ce.schwarz) {
            SchwarzLaunch sl{pnat, prims, didx + cls_off[c], n, dQ};
            if (ce.schwarz(sl, s)) return fail(MJK_ERR_HIP, "mjk_plan_bind: Schwarz launch failed");
            continue;
        }
        // split class: diagonal quartets (AB|AB) through its eri launcher in Schwarz mode
        const StageView st = eri_stage(p);
        std::vector<EriItem> items(n);
        for (int i = 0; i < n; ++i) {
            EriItem it{};
            it.bra = it.ket = p->class_pairs[c][i];
            it.n1 = it.n3 = ncart_h(ce.la);
            it.n2 = it.n4 = ncart_h(ce.lb);
            items[i] = it;
        }
        auto *stage_items = (EriItem *)(w + p->o_eri);
        for (int i0 = 0; i0 < n; i0 += kEriStage) {
            const int m = std::min(kEriStage, n - i0);
            HIP_TRY(hipMemcpyAsync(stage_items, items.data() + i0, sizeof(EriItem) * m, hipMemcpyHostToDevice, s));
            // few quartets, each with up to 6^4 primitive quartets: spread those over the lanes
            EriLaunch el{pnat, prims, stage_items, m, nullptr, st.ptr, st.bytes, st.nslot, dQ, 1};
            const int rc = ce.eri(el, s);
            if (rc == kLaunchStaging)
                return fail(MJK_ERR_STATE, "mjk_plan_bind: Schwarz factors of class (%d%d|%d%d): staging region of "
                            "%zu bytes too small", ce.la, ce.lb, ce.lc, ce.ld, st.bytes);
            if (rc) return fail(MJK_ERR_HIP, "mjk_plan_bind: Schwarz launch failed");
            HIP_TRY(hipStreamSynchronize(s));  // the staged items are rewritten by the next chunk
        }
    }
    p->Q.resize(p->npair);
    HIP_TRY(hipMemcpyAsync(p->Q.data(), dQ, sizeof(double) * p->npair, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < p->npair; ++k) {
        if (!std::isfinite(p->Q[k])) return fail(MJK_ERR_HIP, "mjk_plan_bind: Schwarz factor %d not finite", k);
        p->pairs_nat[k].Q = p->Q[k];
    }

    // sort into bins: (class, K-bucket) ascending, then by first shell (runs),
    // inside a run Q descending, index ascending
    p->sorted.resize(p->npair);
    for (int k = 0; k < p->npair; ++k) p->sorted[k] = k;
    std::stable_sort(p->sorted.begin(), p->sorted.end(), [&](int x, int y) {
        const ShellPairD &a = p->pairs_nat[x], &b = p->pairs_nat[y];
        const bool kbins = !(p->opts.flags & MJK_FLAG_NO_KBINS);
        const int ka = a.cls * kNumKBuckets + (kbins ? kbucket(a.nprim) : 0),
                  kb = b.cls * kNumKBuckets + (kbins ? kbucket(b.nprim) : 0);
        if (ka != kb) return ka < kb;
        if (a.A != b.A) return a.A < b.A;
        if (a.Q != b.Q) return a.Q > b.Q;
        return x < y;
    });
    std::vector<ShellPairD> &psort = p->psort;
    psort.resize(p->npair);
    for (int k = 0; k < p->npair; ++k) psort[k] = p->pairs_nat[p->sorted[k]];
    HIP_TRY(hipMemcpyAsync(w + p->o_psort, psort.data(), sizeof(ShellPairD) * p->npair, hipMemcpyHostToDevice, s));
    // runs of every bin: bin-relative start and length
    auto &bin_runs = p->bin_runs;
    bin_runs.assign(p->bins.size(), {});
    for (size_t y = 0; y < p->bins.size(); ++y) {
        const Bin &Y = p->bins[y];
        auto &rs = bin_runs[y];
        for (int k = 0; k < Y.count; ++k) {
            if (k == 0 || psort[Y.begin + k].A != psort[Y.begin + k - 1].A)
                rs.push_back({k, 1});
            else
                rs.back().second++;
        }
        if ((int)rs.size() != Y.nrun) return fail(MJK_ERR_STATE, "mjk_plan_bind: bin %zu: run count changed since create", y);
    }

    p->dens_screen = false;
    if (int rc = build_lists(p, nullptr, 0.0, s)) return rc;
    p->bound = true;
    return MJK_OK;
}

static int check_density_host(int64_t nbf, const double *D, const char *who)
{
    const size_t n = (size_t)nbf;
    std::vector<double> h(n * n);
    HIP_TRY(hipMemcpy(h.data(), D, sizeof(double) * n * n, hipMemcpyDeviceToHost));
    double mx = 0.0;
    for (double v : h) {
        if (!std::isfinite(v)) return fail(MJK_ERR_INVALID_ARG, "%s: D has a non-finite entry", who);
        mx = std::max(mx, std::fabs(v));
    }
    for (size_t i = 0; i < n; ++i)
        for (size_t j = 0; j < i; ++j)
            if (std::fabs(h[i * n + j] - h[j * n + i]) > 1e-12 * mx)
                return fail(MJK_ERR_INVALID_ARG, "%s: D is not symmetric at (%zu, %zu)", who, i, j);
    return MJK_OK;
}

extern "C" {

int mjk_nbf(const mjk_basis *basis, int64_t *nbf)
{
    if (!nbf) return fail(MJK_ERR_INVALID_ARG, "mjk_nbf: nbf is NULL");
    if (int rc = validate_basis(basis)) return rc;
    int64_t n = 0;
    for (int s = 0; s < basis->nshell; ++s) n += ncart_h(basis->shell_l[s]);
    *nbf = n;
    return MJK_OK;
}

int mjk_plan_create(mjk_ctx *ctx, const mjk_basis *b, const mjk_jk_opts *opts, mjk_plan **out, size_t *ws_bytes)
{
    return plan_create(ctx, b, opts, false, out, ws_bytes);
}

void mjk_plan_destroy(mjk_plan *plan) { delete plan; }

int mjk_plan_bind(mjk_plan *p, void *workspace, size_t bytes, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_bind: plan is NULL");
    CtxScope cs_(p->ctx);
    if (p->in_batch) return fail(MJK_ERR_STATE, "mjk_plan_bind: plan belongs to a batch");
    return plan_bind(p, workspace, bytes, (hipStream_t)stream);
}

int mjk_plan_set_tiles(mjk_plan *p, const int32_t *qpl, int32_t n)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_set_tiles: plan is NULL");
    CtxScope cs_(p->ctx);
    if (!p->bound) return fail(MJK_ERR_STATE, "mjk_plan_set_tiles: plan is not bound");
    int units[kTileUnits];
    if (int rc = check_qpl(qpl, n, "mjk_plan_set_tiles", units)) return rc;
    HIP_TRY(hipSetDevice(p->ctx->device));
    HIP_TRY(hipDeviceSynchronize());  // no launch of this plan may still read the lists
    for (int u = 0; u < kTileUnits; ++u) p->qpl[u] = units[u];
    rechunk(p, -1);
    if (int rc = upload_work(p, nullptr)) return rc;
    p->groups = make_groups({p});
    const int64_t zero = 0;
    return upload_groups(p->groups, {p}, &zero, (JKSeg *)(p->ws + p->o_segs), nullptr);
}

// J and K of one plan with the given work counters and staging region.
static int build_jk_run(mjk_plan *p, const double *D, double *J, double *K, hipStream_t s, uint32_t *queue,
                        double *stage, size_t stage_bytes, int nslot, bool timed, const char *who)
{
    if (!p->bound || p->in_batch) return fail(MJK_ERR_STATE, "%s: plan is not bound", who);
    if (!D || !J || !K) return fail(MJK_ERR_INVALID_ARG, "%s: NULL matrix", who);
    if (J == K || (const double *)J == D || (const double *)K == D)
        return fail(MJK_ERR_INVALID_ARG, "%s: D, J, K must be distinct buffers", who);
    HIP_TRY(hipSetDevice(p->ctx->device));
    if (p->opts.flags & MJK_FLAG_CHECK) {
        HIP_TRY(hipStreamSynchronize(s));
        if (int rc = check_density_host(p->nbf, D, who)) return rc;
    }
    const int64_t n2 = (int64_t)p->nbf * p->nbf;
    if (launch_fill(J, n2, 0.0, s) || launch_fill(K, n2, 0.0, s)) return fail(MJK_ERR_HIP, "%s: fill launch failed", who);
    if (timed)
        if (int rc = ensure_events(p->ev, 2 * p->groups.size())) return rc;
    p->timed_last = timed;
    p->timed_grad = false;
    if (int rc = run_groups(p->groups, (const JKSeg *)(p->ws + p->o_segs), queue, stage, stage_bytes, nslot, D, J, K,
                            nullptr, 0, nullptr, s, timed ? &p->ev : nullptr, who,
                            (p->opts.flags & MJK_FLAG_PERSISTENT) != 0))
        return rc;
    if (launch_symmetrize(J, p->nbf, s) || launch_symmetrize(K, p->nbf, s))
        return fail(MJK_ERR_HIP, "%s: symmetrize launch failed", who);
    return MJK_OK;
}

int mjk_build_jk(mjk_plan *p, const double *D, double *J, double *K, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_build_jk: plan is NULL");
    CtxScope cs_(p->ctx);
    if (p->opts.flags & MJK_FLAG_NO_STAGING)
        return fail(MJK_ERR_STATE, "mjk_build_jk: the plan has no staging (MJK_FLAG_NO_STAGING): use "
                                   "mjk_build_jk_static");
    char *w = p->ws;
    return build_jk_run(p, D, J, K, (hipStream_t)stream, (uint32_t *)(w + p->o_queue), (double *)(w + p->o_stage),
                        p->stage_bytes(), p->nslot, p->timing, "mjk_build_jk");
}

int mjk_build_jk_static(mjk_plan *p, const double *D, double *J, double *K, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_build_jk_static: plan is NULL");
    CtxScope cs_(p->ctx);
    char *scr = p->ctx->scratch;
    if (!scr) return fail(MJK_ERR_STATE, "mjk_build_jk_static: no static scratch on device %d", p->ctx->device);
    // counters: one per launch; staging: as many slots of the plan's stride as fit
    if (sizeof(uint32_t) * 2 * kNumQuartetClasses > kStaticQueueBytes)
        return fail(MJK_ERR_UNSUPPORTED, "mjk_build_jk_static: work counters exceed the static scratch");
    const size_t slot = sizeof(double) * 64 * p->stage_nacc;
    int nslot = 0;
    if (slot > 0) {
        const size_t fit = (kStaticScratchBytes - kStaticQueueBytes) / slot;
        if (fit < 1)
            return fail(MJK_ERR_UNSUPPORTED, "mjk_build_jk_static: one staging slot (%zu bytes) exceeds the static "
                        "scratch (%zu bytes)", slot, kStaticScratchBytes - kStaticQueueBytes);
        nslot = (int)std::min<size_t>(fit, (size_t)p->nslot_max);
    }
    return build_jk_run(p, D, J, K, (hipStream_t)stream, (uint32_t *)scr, (double *)(scr + kStaticQueueBytes),
                        slot * (size_t)nslot, nslot, false, "mjk_build_jk_static");
}

int mjk_e2(mjk_plan *p, const double *D, const double *J, const double *K, double *e2, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_e2: plan is NULL");
    CtxScope cs_(p->ctx);
    if (!D || !J || !K || !e2) return fail(MJK_ERR_INVALID_ARG, "mjk_e2: NULL argument");
    HIP_TRY(hipSetDevice(p->ctx->device));
    if (launch_e2(D, J, K, p->nbf, e2, (hipStream_t)stream)) return fail(MJK_ERR_HIP, "mjk_e2: launch failed");
    return MJK_OK;
}

int mjk_grad_e2(mjk_plan *p, const double *D, double *grad, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_grad_e2: plan is NULL");
    CtxScope cs_(p->ctx);
    if (!p->bound || p->in_batch) return fail(MJK_ERR_STATE, "mjk_grad_e2: plan is not bound");
    if (!(p->opts.flags & MJK_FLAG_GRAD))
        return fail(MJK_ERR_STATE, "mjk_grad_e2: plan was created without MJK_FLAG_GRAD");
    if (!D || !grad) return fail(MJK_ERR_INVALID_ARG, "mjk_grad_e2: NULL argument");
    if (p->natom > kGradMaxAtoms)
        return fail(MJK_ERR_UNSUPPORTED, "mjk_grad_e2: %d atoms > %d", p->natom, kGradMaxAtoms);
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (p->opts.flags & MJK_FLAG_CHECK) {
        HIP_TRY(hipStreamSynchronize(s));
        if (int rc = check_density_host(p->nbf, D, "mjk_grad_e2")) return rc;
    }
    if (launch_fill(grad, 3 * (int64_t)p->natom, 0.0, s)) return fail(MJK_ERR_HIP, "mjk_grad_e2: fill failed");
    char *w = p->ws;
    if (p->timing)
        if (int rc = ensure_events(p->ev, 2 * p->groups.size())) return rc;
    p->timed_last = p->timing;
    p->timed_grad = true;
    return run_groups(p->groups, (const JKSeg *)(w + p->o_segs), (uint32_t *)(w + p->o_queue),
                      (double *)(w + p->o_stage), p->stage_bytes(), p->nslot, D, nullptr, nullptr, grad, p->natom,
                      nullptr, s, p->timing ? &p->ev : nullptr, "mjk_grad_e2");
}

int mjk_e2_backward(mjk_plan *p, const double *D, const double *J, const double *K, const double *gout, double *gD,
                    double *gR, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_e2_backward: plan is NULL");
    CtxScope cs_(p->ctx);
    if (!p->bound || p->in_batch) return fail(MJK_ERR_STATE, "mjk_e2_backward: plan is not bound");
    if (gD && (!J || !K)) return fail(MJK_ERR_INVALID_ARG, "mjk_e2_backward: gD needs J and K");
    if (gD && ((const double *)gD == J || (const double *)gD == K))
        return fail(MJK_ERR_INVALID_ARG, "mjk_e2_backward: gD must not alias J or K");
    if (gR && !D) return fail(MJK_ERR_INVALID_ARG, "mjk_e2_backward: gR needs D");
    if (gR && !(p->opts.flags & MJK_FLAG_GRAD))
        return fail(MJK_ERR_STATE, "mjk_e2_backward: plan was created without MJK_FLAG_GRAD");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (gD && launch_e2_grad_D(J, K, gout, gD, (int64_t)p->nbf * p->nbf, s))
        return fail(MJK_ERR_HIP, "mjk_e2_backward: launch failed");
    if (gR) {
        if (int rc = mjk_grad_e2(p, D, gR, stream)) return rc;
        if (gout && launch_scale(gR, 3 * (int64_t)p->natom, gout, s))
            return fail(MJK_ERR_HIP, "mjk_e2_backward: launch failed");
    }
    return MJK_OK;
}

int mjk_eri_class(mjk_plan *p, const int32_t *quartets, int64_t nq, double *out, int64_t out_len, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_eri_class: plan is NULL");
    CtxScope cs_(p->ctx);
    if (!p->bound) return fail(MJK_ERR_STATE, "mjk_eri_class: plan is not bound");
    if (nq < 0 || (nq > 0 && (!quartets || !out)))
        return fail(MJK_ERR_INVALID_ARG, "mjk_eri_class: bad quartet list");
    // canonicalize and group by quartet class and precision (fp32_tau)
    std::vector<std::vector<EriItem>> groups(2 * kNumQuartetClasses);
    const double tau32 = p->opts.fp32_tau;
    int64_t total = 0;
    for (int64_t q = 0; q < nq; ++q) {
        int sh[4];
        for (int k = 0; k < 4; ++k) {
            sh[k] = quartets[4 * q + k];
            if (sh[k] < 0 || sh[k] >= p->nshell)
                return fail(MJK_ERR_INVALID_ARG, "mjk_eri_class: quartet %lld shell %d out of range", (long long)q,
                            sh[k]);
        }
        auto pidx = [](int a, int b) { return std::max(a, b) * (std::max(a, b) + 1) / 2 + std::min(a, b); };
        const int P = pidx(sh[0], sh[1]), Qp = pidx(sh[2], sh[3]);
        const ShellPairD &pp = p->pairs_nat[P], &pq = p->pairs_nat[Qp];
        EriItem it{};
        int flags = 0;
        if (pp.A != sh[0]) flags |= 1;  // caller's (A, B) is the pair's (second, first)
        if (pq.A != sh[2]) flags |= 2;
        int bra = P, ket = Qp;
        if (pp.cls < pq.cls) {
            std::swap(bra, ket);
            flags |= 4;
        }
        it.bra = bra;
        it.ket = ket;
        it.flags = flags;
        it.out_off = total;
        it.n1 = ncart_h(p->l[sh[0]]);
        it.n2 = ncart_h(p->l[sh[1]]);
        it.n3 = ncart_h(p->l[sh[2]]);
        it.n4 = ncart_h(p->l[sh[3]]);
        total += (int64_t)it.n1 * it.n2 * it.n3 * it.n4;
        const int qc = quartet_class(p->pairs_nat[bra].cls, p->pairs_nat[ket].cls);
        const bool f32 = tau32 > 0.0 && fp32_allowed(kClassTable[qc]) && p->Q[bra] * p->Q[ket] < tau32;
        groups[2 * qc + (f32 ? 1 : 0)].push_back(it);
    }
    if (total != out_len)
        return fail(MJK_ERR_INVALID_ARG, "mjk_eri_class: out_len %lld, quartets need %lld", (long long)out_len,
                    (long long)total);
    if (nq == 0) return MJK_OK;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    char *w = p->ws;
    auto *stage = (EriItem *)(w + p->o_eri);
    for (int gi = 0; gi < 2 * kNumQuartetClasses; ++gi) {
        const int qc = gi / 2;
        const auto &g = groups[gi];
        for (size_t i0 = 0; i0 < g.size(); i0 += kEriStage) {
            const int n = (int)std::min<size_t>(kEriStage, g.size() - i0);
            // stream order keeps this copy behind the previous launch that read the stage
            HIP_TRY(hipMemcpyAsync(stage, g.data() + i0, sizeof(EriItem) * n, hipMemcpyHostToDevice, s));
            const StageView st = eri_stage(p);
            // split classes: few requested quartets run one per block, primitive quartets over the lanes
            EriLaunch a{(const ShellPairD *)(w + p->o_pnat), (const PrimPairD *)(w + p->o_prims), stage, n, out,
                        st.ptr, st.bytes, st.nslot, nullptr, n <= kEriDeconstructMax ? 1 : 0};
            const int rc = (gi % 2 ? kClassTable[qc].eri32 : kClassTable[qc].eri)(a, s);
            if (rc == kLaunchStaging)
                return fail(MJK_ERR_STATE, "mjk_eri_class: staging region of %zu bytes too small for class %d",
                            st.bytes, qc);
            if (rc) return fail(MJK_ERR_HIP, "mjk_eri_class: launch failed");
            HIP_TRY(hipStreamSynchronize(s));  // the host vector g is pageable and reused
        }
    }
    return MJK_OK;
}

int mjk_plan_set_density_screen(mjk_plan *p, const double *dD, double tau, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_set_density_screen: plan is NULL");
    CtxScope cs_(p->ctx);
    if (!p->bound || p->in_batch) return fail(MJK_ERR_STATE, "mjk_plan_set_density_screen: plan is not bound");
    if (dD && !(std::isfinite(tau) && tau >= 0.0))
        return fail(MJK_ERR_INVALID_ARG, "mjk_plan_set_density_screen: tau = %g", tau);
    if (!dD && !p->dens_screen) return MJK_OK;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> shell_w;
    if (dD) {
        // largest |dD| of every AO row, then of every shell's rows
        std::vector<double> row(p->nbf);
        if (launch_rowmax_abs(dD, p->nbf, (double *)(p->ws + p->o_rowmax), s))
            return fail(MJK_ERR_HIP, "mjk_plan_set_density_screen: launch failed");
        HIP_TRY(hipMemcpyAsync(row.data(), p->ws + p->o_rowmax, sizeof(double) * p->nbf, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        shell_w.assign(p->nshell, 0.0);
        for (int A = 0; A < p->nshell; ++A)
            for (int a = 0; a < ncart_h(p->l[A]); ++a) {
                const double v = row[p->ao[A] + a];
                if (!std::isfinite(v))
                    return fail(MJK_ERR_INVALID_ARG, "mjk_plan_set_density_screen: dD has a non-finite entry");
                shell_w[A] = std::max(shell_w[A], v);
            }
    }
    HIP_TRY(hipDeviceSynchronize());  // no launch of this plan may still read the lists
    if (int rc = build_lists(p, dD ? shell_w.data() : nullptr, tau, s)) return rc;
    p->dens_screen = dD != nullptr;
    return MJK_OK;
}

int mjk_one_electron(mjk_plan *p, const double *Z, double *S, double *T, double *V, double *enuc, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_one_electron: plan is NULL");
    CtxScope cs_(p->ctx);
    if (!p->bound || p->in_batch) return fail(MJK_ERR_STATE, "mjk_one_electron: plan is not bound");
    if (!Z) return fail(MJK_ERR_INVALID_ARG, "mjk_one_electron: Z is NULL");
    if (!S && !T && !V && !enuc) return MJK_OK;
    if ((S && (S == T || S == V)) || (T && T == V))
        return fail(MJK_ERR_INVALID_ARG, "mjk_one_electron: S, T, V must be distinct");
    HIP_TRY(hipSetDevice(p->ctx->device));
    char *w = p->ws;
    if (launch_one_electron((const ShellPairD *)(w + p->o_pnat), (const PrimPairD *)(w + p->o_prims),
                            (const int32_t *)(w + p->o_cls), p->class_off.data(), kLmax,
                            (const double *)(w + p->o_xyz), Z, p->natom, p->nbf, S, T, V, enuc,
                            (hipStream_t)stream))
        return fail(MJK_ERR_HIP, "mjk_one_electron: launch failed");
    return MJK_OK;
}

int mjk_schwarz(mjk_plan *p, double *Qh)
{
    if (!p || !Qh) return fail(MJK_ERR_INVALID_ARG, "mjk_schwarz: NULL argument");
    CtxScope cs_(p->ctx);
    if (!p->bound) return fail(MJK_ERR_STATE, "mjk_schwarz: plan is not bound");
    const int ns = p->nshell;
    for (int A = 0, k = 0; A < ns; ++A)
        for (int B = 0; B <= A; ++B, ++k) Qh[A * ns + B] = Qh[B * ns + A] = p->Q[k];
    return MJK_OK;
}

int mjk_plan_set_timing(mjk_plan *p, int enable)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_set_timing: plan is NULL");
    CtxScope cs_(p->ctx);
    p->timing = enable != 0;
    return MJK_OK;
}

int mjk_plan_timings(mjk_plan *p, mjk_class_timing *out, int32_t cap, int32_t *n)
{
    if (!p || !n || (cap > 0 && !out)) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_timings: NULL argument");
    CtxScope cs_(p->ctx);
    if (!p->timed_last || p->ev.size() != 2 * p->groups.size())
        return fail(MJK_ERR_STATE, "mjk_plan_timings: the last build ran without timing");
    return fill_timings(p->groups, p->ev, p->timed_grad, out, cap, n);
}

int mjk_plan_stats_get(const mjk_plan *p, mjk_plan_stats *st)
{
    if (!p || !st) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_stats_get: NULL argument");
    *st = p->stats;
    return MJK_OK;
}

// ---------------------------------------------------------------------------
// Batches: many molecules, one launch per (class, precision) over all of them
// ---------------------------------------------------------------------------

int mjk_batch_create(mjk_ctx *ctx, int32_t nmol, const mjk_basis *mols, const mjk_jk_opts *opts, mjk_batch **out,
                     size_t *ws_bytes)
{
    if (!ctx || !mols || !out || !ws_bytes) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_create: NULL argument");
    CtxScope cs_(ctx);
    *out = nullptr;
    if (nmol <= 0) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_create: nmol = %d", nmol);
    if (opts && (opts->flags & MJK_FLAG_GRAD))
        return fail(MJK_ERR_INVALID_ARG, "mjk_batch_create: batches build J and K only (no MJK_FLAG_GRAD)");
    auto *bt = new mjk_batch;
    bt->ctx = ctx;
    for (int q = 0; q < kNumQuartetClasses * kNumKBuckets; ++q) bt->qpl[q] = 1;
    size_t off = 0;
    int64_t moff = 0, max_items = 0;
    bt->mat_off.push_back(0);
    for (int m = 0; m < nmol; ++m) {
        mjk_plan *p = nullptr;
        size_t bytes = 0;
        if (int rc = plan_create(ctx, &mols[m], opts, true, &p, &bytes)) {
            delete bt;
            const std::string why = g_err;
            return fail(rc, "mjk_batch_create: molecule %d: %s", m, why.c_str());
        }
        bt->plans.push_back(p);
        bt->ws_off.push_back(off);
        off = align_up(off + bytes);
        moff += (int64_t)p->nbf * p->nbf;
        bt->mat_off.push_back(moff);
        bt->nseg += p->lists.size();
        bt->stage_nacc = std::max(bt->stage_nacc, p->stage_nacc);
        max_items += p->max_items;
    }
    bt->nslot = bt->stage_nacc ? (int)std::min<int64_t>(kSlotsPerCU * std::max(1, ctx->ncu), 2 * max_items) : 0;
    auto take = [&](size_t bytes) {
        const size_t o2 = off;
        off = align_up(off + bytes);
        return o2;
    };
    bt->o_segs = take(sizeof(JKSeg) * bt->nseg);
    bt->o_queue = take(sizeof(uint32_t) * 2 * kNumQuartetClasses);
    bt->o_stamps = take(sizeof(unsigned long long) * 2 * nmol);
    bt->o_stage = take(bt->stage_bytes());
    bt->total = off;
    *ws_bytes = off;
    *out = bt;
    return MJK_OK;
}

void mjk_batch_destroy(mjk_batch *b) { delete b; }

static int batch_regroup(mjk_batch *b, hipStream_t s)
{
    b->groups = make_groups(b->plans);
    return upload_groups(b->groups, b->plans, b->mat_off.data(), (JKSeg *)(b->ws + b->o_segs), s);
}

int mjk_batch_bind(mjk_batch *b, void *workspace, size_t bytes, void *stream)
{
    if (!b) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_bind: batch is NULL");
    CtxScope cs_(b->ctx);
    if (!workspace) return fail(MJK_ERR_WORKSPACE, "mjk_batch_bind: workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(MJK_ERR_WORKSPACE, "mjk_batch_bind: workspace not 256-byte aligned");
    if (bytes < b->total)
        return fail(MJK_ERR_WORKSPACE, "mjk_batch_bind: workspace %zu bytes < %zu needed", bytes, b->total);
    b->bound = false;
    b->ws = (char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    for (size_t m = 0; m < b->plans.size(); ++m) {
        mjk_plan *p = b->plans[m];
        for (int q = 0; q < kNumQuartetClasses * kNumKBuckets; ++q) p->qpl[q] = b->qpl[q];
        // the batch's staging serves the molecule's Schwarz factors (binds are
        // synchronous, so the molecules take it in turn)
        p->lent_stage = (double *)(b->ws + b->o_stage);
        p->lent_stage_bytes = b->stage_bytes();
        p->lent_nslot = b->nslot;
        const int rc = plan_bind(p, b->ws + b->ws_off[m], p->total, s);
        p->lent_stage = nullptr;
        p->lent_stage_bytes = 0;
        p->lent_nslot = 0;
        if (rc) return rc;
    }
    if (int rc = batch_regroup(b, s)) return rc;
    b->bound = true;
    return MJK_OK;
}

int mjk_batch_offsets(const mjk_batch *b, int64_t *mat_off)
{
    if (!b || !mat_off) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_offsets: NULL argument");
    for (size_t m = 0; m < b->mat_off.size(); ++m) mat_off[m] = b->mat_off[m];
    return MJK_OK;
}

int mjk_batch_set_tiles(mjk_batch *b, const int32_t *qpl, int32_t n)
{
    if (!b) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_set_tiles: batch is NULL");
    CtxScope cs_(b->ctx);
    if (!b->bound) return fail(MJK_ERR_STATE, "mjk_batch_set_tiles: batch is not bound");
    int units[kTileUnits];
    if (int rc = check_qpl(qpl, n, "mjk_batch_set_tiles", units)) return rc;
    HIP_TRY(hipSetDevice(b->ctx->device));
    HIP_TRY(hipDeviceSynchronize());  // no launch of this batch may still read the lists
    for (int u = 0; u < kTileUnits; ++u) b->qpl[u] = units[u];
    for (auto *p : b->plans) {
        for (int u = 0; u < kTileUnits; ++u) p->qpl[u] = units[u];
        rechunk(p, -1);
        if (int rc = upload_work(p, nullptr)) return rc;
    }
    return batch_regroup(b, nullptr);
}

int mjk_batch_set_stamps(mjk_batch *b, int enable)
{
    if (!b) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_set_stamps: batch is NULL");
    CtxScope cs_(b->ctx);
    b->stamps = enable != 0;
    return MJK_OK;
}

int mjk_batch_set_timing(mjk_batch *b, int enable)
{
    if (!b) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_set_timing: batch is NULL");
    CtxScope cs_(b->ctx);
    b->timing = enable != 0;
    return MJK_OK;
}

static int batch_run(mjk_batch *b, const double *D, double *J, double *K, hipStream_t s, bool timed)
{
    if (timed)
        if (int rc = ensure_events(b->ev, 2 * b->groups.size())) return rc;
    unsigned long long *st = nullptr;
    if (b->stamps) {
        st = (unsigned long long *)(b->ws + b->o_stamps);
        if (launch_stamp_init(st, (int)b->plans.size(), s)) return fail(MJK_ERR_HIP, "mjk_batch_build_jk: stamp init");
    }
    b->stamped_last = b->stamps;
    return run_groups(b->groups, (const JKSeg *)(b->ws + b->o_segs), (uint32_t *)(b->ws + b->o_queue),
                      (double *)(b->ws + b->o_stage), b->stage_bytes(), b->nslot, D, J, K, nullptr, 0, st, s,
                      timed ? &b->ev : nullptr, "mjk_batch_build_jk",
                      (b->plans[0]->opts.flags & MJK_FLAG_PERSISTENT) != 0);
}

int mjk_batch_build_jk(mjk_batch *b, const double *D, double *J, double *K, void *stream)
{
    if (!b) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_build_jk: batch is NULL");
    CtxScope cs_(b->ctx);
    if (!b->bound) return fail(MJK_ERR_STATE, "mjk_batch_build_jk: batch is not bound");
    if (!D || !J || !K) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_build_jk: NULL matrix");
    if (J == K || (const double *)J == D || (const double *)K == D)
        return fail(MJK_ERR_INVALID_ARG, "mjk_batch_build_jk: D, J, K must be distinct buffers");
    HIP_TRY(hipSetDevice(b->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t tot = b->mat_off.back();
    if (launch_fill(J, tot, 0.0, s) || launch_fill(K, tot, 0.0, s))
        return fail(MJK_ERR_HIP, "mjk_batch_build_jk: fill launch failed");
    b->timed_last = b->timing;
    if (int rc = batch_run(b, D, J, K, s, b->timing)) return rc;
    for (size_t m = 0; m < b->plans.size(); ++m) {
        const int n = b->plans[m]->nbf;
        if (launch_symmetrize(J + b->mat_off[m], n, s) || launch_symmetrize(K + b->mat_off[m], n, s))
            return fail(MJK_ERR_HIP, "mjk_batch_build_jk: symmetrize launch failed");
    }
    return MJK_OK;
}

int mjk_batch_timings(mjk_batch *b, mjk_class_timing *out, int32_t cap, int32_t *n)
{
    if (!b || !n || (cap > 0 && !out)) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_timings: NULL argument");
    CtxScope cs_(b->ctx);
    if (!b->timed_last || b->ev.size() != 2 * b->groups.size())
        return fail(MJK_ERR_STATE, "mjk_batch_timings: the last build ran without timing");
    return fill_timings(b->groups, b->ev, false, out, cap, n);
}

int mjk_batch_mol_times(mjk_batch *b, double *ms)
{
    if (!b || !ms) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_mol_times: NULL argument");
    CtxScope cs_(b->ctx);
    if (!b->stamped_last) return fail(MJK_ERR_STATE, "mjk_batch_mol_times: the last build ran without stamps");
    const size_t nm = b->plans.size();
    std::vector<unsigned long long> h(2 * nm);
    HIP_TRY(hipSetDevice(b->ctx->device));
    HIP_TRY(hipMemcpy(h.data(), b->ws + b->o_stamps, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->ctx->device));
    if (khz <= 0) return fail(MJK_ERR_HIP, "mjk_batch_mol_times: wall clock rate unknown");
    unsigned long long t0 = ~0ull;
    for (size_t m = 0; m < nm; ++m)
        if (h[2 * m + 1] != 0) t0 = std::min(t0, h[2 * m]);
    for (size_t m = 0; m < nm; ++m) {
        if (h[2 * m + 1] == 0) {  // no work in this molecule
            ms[2 * m] = ms[2 * m + 1] = 0.0;
            continue;
        }
        ms[2 * m] = (double)(h[2 * m] - t0) / khz;
        ms[2 * m + 1] = (double)(h[2 * m + 1] - t0) / khz;
    }
    return MJK_OK;
}

int mjk_batch_stats(const mjk_batch *b, mjk_plan_stats *total, int64_t *nq_per_mol)
{
    if (!b || !total) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_stats: NULL argument");
    if (!b->bound) return fail(MJK_ERR_STATE, "mjk_batch_stats: batch is not bound");
    mjk_plan_stats t{};
    for (size_t m = 0; m < b->plans.size(); ++m) {
        const mjk_plan_stats &s = b->plans[m]->stats;
        t.nbf += s.nbf;
        t.nshell += s.nshell;
        t.npair += s.npair;
        t.nprim_pair += s.nprim_pair;
        t.nquartet_total += s.nquartet_total;
        t.nquartet_kept += s.nquartet_kept;
        t.nquartet_fp32 += s.nquartet_fp32;
        t.nprim_quartet_kept += s.nprim_quartet_kept;
        t.ncart_eri_kept += s.ncart_eri_kept;
        t.vrr_flops_kept += s.vrr_flops_kept;
        if (nq_per_mol) nq_per_mol[m] = s.nquartet_kept;
    }
    t.nlaunch = (int64_t)b->groups.size() + 2 + 2 * (int64_t)b->plans.size();
    t.workspace_bytes = b->total;
    *total = t;
    return MJK_OK;
}

// Algorithm 2: every class starts at one quartet per lane; in each sweep a
// class is timed, its workload doubled (Combine), timed again, and kept if
// faster, else halved back (Revert); sweeps repeat while any class improved.
// Times are the shortest of `reps` launches of that class alone.  J and K
// hold no meaningful values afterwards.
int mjk_batch_autotune(mjk_batch *b, const double *D, double *J, double *K, int32_t reps, int32_t *qpl,
                       int32_t n, void *stream)
{
    if (!b) return fail(MJK_ERR_INVALID_ARG, "mjk_batch_autotune: batch is NULL");
    CtxScope cs_(b->ctx);
    if (!b->bound) return fail(MJK_ERR_STATE, "mjk_batch_autotune: batch is not bound");
    if (!D || !J || !K || !qpl || (n != kNumQuartetClasses && n != kTileUnits) || reps < 1)
        return fail(MJK_ERR_INVALID_ARG, "mjk_batch_autotune: bad argument");
    // entries 0 mark the units to tune (they start at 1); the others are fixed
    std::vector<int32_t> start(n);
    std::vector<bool> tune(n);
    for (int i = 0; i < n; ++i) {
        tune[i] = qpl[i] == 0;
        start[i] = tune[i] ? 1 : qpl[i];
    }
    int units_now[kTileUnits];
    if (int rc = check_qpl(start.data(), n, "mjk_batch_autotune", units_now)) return rc;
    HIP_TRY(hipSetDevice(b->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int per = n == kTileUnits ? 1 : kNumKBuckets;  // table entries -> units
    const bool stamps = b->stamps;
    b->stamps = false;
    std::vector<int32_t> cur(start);
    if (int rc = mjk_batch_set_tiles(b, cur.data(), n)) return rc;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const bool persistent = (b->plans[0]->opts.flags & MJK_FLAG_PERSISTENT) != 0;
    // the objective of an entry is the time of its class's launches alone
    auto time_class = [&](int q, double &best) -> int {
        std::vector<Group> sel;
        for (const auto &g : b->groups)
            if (g.qcls == q) sel.push_back(g);
        best = 1e300;
        for (int r = 0; r < reps; ++r) {
            HIP_TRY(hipEventRecord(e0, s));
            if (int rc = run_groups(sel, (const JKSeg *)(b->ws + b->o_segs), (uint32_t *)(b->ws + b->o_queue),
                                    (double *)(b->ws + b->o_stage), b->stage_bytes(), b->nslot, D, J, K, nullptr, 0,
                                    nullptr, s, nullptr, "mjk_batch_autotune", persistent))
                return rc;
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, (double)ms);
        }
        return MJK_OK;
    };
    // entries to tune that have work: their class has launches (and, per
    // K-bucket, a bra bin of that bucket with items)
    std::vector<bool> has_work(n, false);
    for (const auto *p : b->plans)
        for (const auto &wl : p->lists) {
            if (wl.nitems == 0) continue;
            const BinPair &bp = p->bps[wl.bp];
            const int e = n == kTileUnits ? bp.qcls * kNumKBuckets + p->bins[bp.X].kb : bp.qcls;
            has_work[e] = true;
        }
    // Algorithm 2: Combine (double the entry's quartets per lane), keep it if
    // its class got faster, else Revert and retire the entry; sweep while any
    // entry improved
    std::vector<bool> done(n, false);
    bool improved = true;
    int rc = MJK_OK;
    while (improved && rc == MJK_OK) {
        improved = false;
        for (int i = 0; i < n && rc == MJK_OK; ++i) {
            if (!tune[i] || !has_work[i] || done[i] || cur[i] >= kMaxQpl) continue;
            const int q = i * per / kNumKBuckets;
            double t1 = 0.0, t2 = 0.0;
            if ((rc = time_class(q, t1))) break;
            cur[i] *= 2;  // Combine
            if ((rc = mjk_batch_set_tiles(b, cur.data(), n))) break;
            if ((rc = time_class(q, t2))) break;
            if (t2 < t1) {
                improved = true;
            } else {
                cur[i] /= 2;  // Revert
                done[i] = true;
                if ((rc = mjk_batch_set_tiles(b, cur.data(), n))) break;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->stamps = stamps;
    if (rc) return rc;
    for (int i = 0; i < n; ++i) qpl[i] = cur[i];
    return MJK_OK;
}

int mjk_num_kbuckets(void) { return kNumKBuckets; }

}  // extern "C"
