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
//            Q_AB Q_CD >= tau), cut into chunks of 64 kets, one wave each.
// Quartets themselves are never stored: only per-bra prefix lengths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mjk.h"
#include "gen/dispatch.inc"
#include "mjk_types.hpp"

namespace mjk {
int launch_pair_table(const ShellPairD *pairs, int npair, const double *xyz, const int32_t *atom,
                      const int32_t *prim_off, const int32_t *nprim, const double *exps, const double *coefs,
                      PrimPairD *out, int nprim_pair, hipStream_t s);
int launch_fill(double *x, int64_t n, double v, hipStream_t s);
int launch_symmetrize(double *M, int n, hipStream_t s);
}  // namespace mjk

using namespace mjk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

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
constexpr int kChunk = 64;          // kets per work item (one per lane)
constexpr int kEriStage = 65536;    // eri_class items per upload
constexpr int kSlotsPerCU = 8;      // resident waves per CU the staging is sized for

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Bin {
    int cls, kb;
    int begin, count;  // positions in the sorted pair order
};

struct BinPair {
    int X, Y;          // bin indices, X >= Y in (class, bucket) order
    int qcls;          // quartet class index
};

// One launch: the FP64 or the FP32 part of one bin pair's quartets.
struct WorkList {
    int bp;            // bin pair
    int fp32;          // 1: FP32 recurrence (Q_AB Q_CD < fp32_tau)
    size_t off;        // int offset in the work-list region:
                       //   ket_start[nbra], ket_end[nbra], chunk_prefix[nbra + 1]
    int nitems;
    int64_t nq;        // kept quartets
    int64_t npq;       // kept primitive quartets
    double cost;       // algorithmic flops
};

// flops per primitive quartet outside the vertical recurrence: geometry (26),
// Boys (Taylor 4(K-1) + 2, downward 3L) and prefactor scaling (L+1)
inline double prim_overhead_flops(int L) { return 26.0 + 4.0 * 7 + 2.0 + 3.0 * L + (L + 1); }

}  // namespace

struct mjk_ctx {
    int device;
    std::string arch;
    int ncu;
};

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
    std::vector<WorkList> lists;
    std::vector<std::vector<int32_t>> class_pairs;  // natural indices per pair class
    // workspace layout (byte offsets)
    size_t o_xyz, o_atom, o_poff, o_np, o_exps, o_coefs, o_pnat, o_psort, o_prims, o_Q, o_cls, o_work, o_eri,
        o_stage, total;
    int nslot = 0;            // staging slots for split classes
    size_t stage_nacc = 0;    // largest split-class accumulator count present
    size_t work_ints = 0;
    char *ws = nullptr;
    bool bound = false;
    mjk_plan_stats stats{};
    // optional per-launch timing
    bool timing = false, timed_last = false;
    std::vector<hipEvent_t> ev;  // 2 per bin pair
    ~mjk_plan()
    {
        for (auto e : ev) hipEventDestroy(e);
    }
};

extern "C" {

int mjk_lmax(void) { return kLmax; }

const char *mjk_last_error(void) { return g_err.c_str(); }

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
        return fail(MJK_ERR_NO_DEVICE, "mjk_ctx_create: device %d is %s, this build targets gfx950", device,
                    arch.c_str());
    auto *c = new mjk_ctx;
    c->device = device;
    c->arch = arch;
    c->ncu = prop.multiProcessorCount;
    *out = c;
    return MJK_OK;
}

void mjk_ctx_destroy(mjk_ctx *ctx) { delete ctx; }

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
    if (!ctx || !out || !ws_bytes) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: NULL argument");
    *out = nullptr;
    if (int rc = validate_basis(b)) return rc;
    mjk_jk_opts o{};
    if (opts) o = *opts;
    if (!(std::isfinite(o.schwarz_tau) && o.schwarz_tau >= 0.0))
        return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: schwarz_tau = %g", o.schwarz_tau);
    if (!(std::isfinite(o.fp32_tau) && o.fp32_tau >= 0.0))
        return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: fp32_tau = %g", o.fp32_tau);
    if (o.flags & ~MJK_FLAG_CHECK) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_create: unknown flags 0x%x", o.flags);

    auto *p = new mjk_plan;
    p->ctx = ctx;
    p->opts = o;
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

    // bins by (class, K-bucket): sizes known now, Q order decided at bind
    std::vector<int> bin_size(kNumPairClasses * kNumKBuckets, 0);
    for (const auto &sp : p->pairs_nat) bin_size[sp.cls * kNumKBuckets + kbucket(sp.nprim)]++;
    int pos = 0;
    for (int c = 0; c < kNumPairClasses; ++c)
        for (int kb = 0; kb < kNumKBuckets; ++kb) {
            const int n = bin_size[c * kNumKBuckets + kb];
            if (n == 0) continue;
            p->bins.push_back({c, kb, pos, n});
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
                woff += 3 * (size_t)p->bins[X].count + 1;
                p->lists.push_back(wl);
            }
            p->bps.push_back(bp);
        }
    p->work_ints = woff;
    // split classes present: staging for one item per persistent block
    for (const auto &bp : p->bps) {
        const ClassEntry &ce = kClassTable[bp.qcls];
        if (ce.split) p->stage_nacc = std::max(p->stage_nacc, (size_t)ce.nacc);
    }
    p->nslot = p->stage_nacc ? kSlotsPerCU * std::max(1, ctx->ncu) : 0;

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
    p->o_eri = take(sizeof(EriItem) * kEriStage);
    p->o_stage = take(sizeof(double) * 64 * p->stage_nacc * (size_t)p->nslot);
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

void mjk_plan_destroy(mjk_plan *plan) { delete plan; }

int mjk_plan_bind(mjk_plan *p, void *workspace, size_t bytes, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_bind: plan is NULL");
    if (!workspace) return fail(MJK_ERR_WORKSPACE, "mjk_plan_bind: workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(MJK_ERR_WORKSPACE, "mjk_plan_bind: workspace not 256-byte aligned");
    if (bytes < p->total)
        return fail(MJK_ERR_WORKSPACE, "mjk_plan_bind: workspace %zu bytes < %zu needed", bytes, p->total);
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
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
    auto *didx = (int32_t *)(w + p->o_cls);
    HIP_TRY(hipMemcpyAsync(didx, cls_idx.data(), sizeof(int32_t) * cls_idx.size(), hipMemcpyHostToDevice, s));
    for (int q = 0; q < kNumQuartetClasses; ++q) {
        const ClassEntry &ce = kClassTable[q];
        if (!ce.schwarz) continue;
        const int c = pair_class(ce.la, ce.lb);
        SchwarzLaunch sl{pnat, prims, didx + cls_off[c], (int32_t)(cls_off[c + 1] - cls_off[c]), dQ};
        if (ce.schwarz(sl, s)) return fail(MJK_ERR_HIP, "mjk_plan_bind: Schwarz launch failed");
    }
    p->Q.resize(p->npair);
    HIP_TRY(hipMemcpyAsync(p->Q.data(), dQ, sizeof(double) * p->npair, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < p->npair; ++k) {
        if (!std::isfinite(p->Q[k])) return fail(MJK_ERR_HIP, "mjk_plan_bind: Schwarz factor %d not finite", k);
        p->pairs_nat[k].Q = p->Q[k];
    }

    // sort into bins: (class, K-bucket) ascending, Q descending, index ascending
    p->sorted.resize(p->npair);
    for (int k = 0; k < p->npair; ++k) p->sorted[k] = k;
    std::stable_sort(p->sorted.begin(), p->sorted.end(), [&](int x, int y) {
        const ShellPairD &a = p->pairs_nat[x], &b = p->pairs_nat[y];
        const int ka = a.cls * kNumKBuckets + kbucket(a.nprim), kb = b.cls * kNumKBuckets + kbucket(b.nprim);
        if (ka != kb) return ka < kb;
        if (a.Q != b.Q) return a.Q > b.Q;
        return x < y;
    });
    std::vector<ShellPairD> psort(p->npair);
    for (int k = 0; k < p->npair; ++k) psort[k] = p->pairs_nat[p->sorted[k]];
    HIP_TRY(hipMemcpyAsync(w + p->o_psort, psort.data(), sizeof(ShellPairD) * p->npair, hipMemcpyHostToDevice, s));

    // stage 2: per bin pair, per bra, the kept ket prefix of the ket bin
    // (Q_AB Q_CD >= schwarz_tau), split into its FP64 prefix
    // (Q_AB Q_CD >= fp32_tau) and FP32 remainder, each cut into chunks
    const double tau = p->opts.schwarz_tau, tau32 = p->opts.fp32_tau;
    std::vector<int32_t> work(p->work_ints, 0);
    int64_t nq_kept = 0, nprimq = 0, ncart = 0, nq32 = 0;
    double flops = 0.0;
    int nlaunch = 0;
    auto prefix_len = [&](const Bin &Y, double qb, double thr) {
        int lo = 0, hi = Y.count;  // first k with qb * Q_k < thr
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (qb * psort[Y.begin + mid].Q < thr)
                hi = mid;
            else
                lo = mid + 1;
        }
        return lo;
    };
    for (size_t il = 0; il < p->lists.size(); il += 2) {
        WorkList &l64 = p->lists[il], &l32 = p->lists[il + 1];
        const BinPair &bp = p->bps[l64.bp];
        const Bin &X = p->bins[bp.X], &Y = p->bins[bp.Y];
        const ClassEntry &ce = kClassTable[bp.qcls];
        int32_t *s64 = work.data() + l64.off, *e64 = s64 + X.count, *p64 = e64 + X.count;
        int32_t *s32 = work.data() + l32.off, *e32 = s32 + X.count, *p32 = e32 + X.count;
        p64[0] = p32[0] = 0;
        std::vector<int64_t> ynp(Y.count + 1, 0);  // prefix of K_C K_D over the ket bin
        for (int k = 0; k < Y.count; ++k) ynp[k + 1] = ynp[k] + psort[Y.begin + k].nprim;
        int64_t q64 = 0, q32 = 0, pq64 = 0, pq32 = 0;
        for (int b = 0; b < X.count; ++b) {
            const double qb = psort[X.begin + b].Q;
            int keep = prefix_len(Y, qb, tau);
            if (bp.X == bp.Y) keep = std::min(keep, b + 1);
            int c64 = tau32 > 0.0 ? std::min(keep, prefix_len(Y, qb, tau32)) : keep;
            s64[b] = 0;
            e64[b] = c64;
            s32[b] = c64;
            e32[b] = keep;
            p64[b + 1] = p64[b] + (c64 + kChunk - 1) / kChunk;
            p32[b + 1] = p32[b] + (keep - c64 + kChunk - 1) / kChunk;
            const int64_t nb = psort[X.begin + b].nprim;
            q64 += c64;
            q32 += keep - c64;
            pq64 += nb * ynp[c64];
            pq32 += nb * (ynp[keep] - ynp[c64]);
        }
        const int nout = ncart_h(ce.la) * ncart_h(ce.lb) * ncart_h(ce.lc) * ncart_h(ce.ld);
        const int L = ce.la + ce.lb + ce.lc + ce.ld;
        const double fpq = ce.vrr_flops + prim_overhead_flops(L), fq = ce.hrr_flops + 12.0 * nout;
        l64.nitems = p64[X.count];
        l64.nq = q64;
        l64.npq = pq64;
        l64.cost = (double)pq64 * fpq + (double)q64 * fq;
        l32.nitems = p32[X.count];
        l32.nq = q32;
        l32.npq = pq32;
        l32.cost = (double)pq32 * fpq + (double)q32 * fq;
        nq_kept += q64 + q32;
        nq32 += q32;
        nprimq += pq64 + pq32;
        ncart += (q64 + q32) * nout;
        flops += l64.cost + l32.cost;
        nlaunch += (l64.nitems > 0) + (l32.nitems > 0);
    }
    if (!work.empty())
        HIP_TRY(hipMemcpyAsync(w + p->o_work, work.data(), sizeof(int32_t) * work.size(), hipMemcpyHostToDevice, s));
    // costliest launches first
    std::stable_sort(p->lists.begin(), p->lists.end(),
                     [](const WorkList &a, const WorkList &b) { return a.cost > b.cost; });
    HIP_TRY(hipStreamSynchronize(s));  // host vectors above are released on return
    p->stats.nquartet_kept = nq_kept;
    p->stats.nquartet_fp32 = nq32;
    p->stats.nprim_quartet_kept = nprimq;
    p->stats.ncart_eri_kept = ncart;
    p->stats.vrr_flops_kept = flops;
    p->stats.nlaunch = nlaunch + 3;
    p->bound = true;
    return MJK_OK;
}

static int check_density_host(const mjk_plan *p, const double *D)
{
    const size_t n = (size_t)p->nbf;
    std::vector<double> h(n * n);
    HIP_TRY(hipMemcpy(h.data(), D, sizeof(double) * n * n, hipMemcpyDeviceToHost));
    double mx = 0.0;
    for (double v : h) {
        if (!std::isfinite(v)) return fail(MJK_ERR_INVALID_ARG, "mjk_build_jk: D has a non-finite entry");
        mx = std::max(mx, std::fabs(v));
    }
    for (size_t i = 0; i < n; ++i)
        for (size_t j = 0; j < i; ++j)
            if (std::fabs(h[i * n + j] - h[j * n + i]) > 1e-12 * mx)
                return fail(MJK_ERR_INVALID_ARG, "mjk_build_jk: D is not symmetric at (%zu, %zu)", i, j);
    return MJK_OK;
}

int mjk_build_jk(mjk_plan *p, const double *D, double *J, double *K, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_build_jk: plan is NULL");
    if (!p->bound) return fail(MJK_ERR_STATE, "mjk_build_jk: plan is not bound");
    if (!D || !J || !K) return fail(MJK_ERR_INVALID_ARG, "mjk_build_jk: NULL matrix");
    if (J == K || (const double *)J == D || (const double *)K == D)
        return fail(MJK_ERR_INVALID_ARG, "mjk_build_jk: D, J, K must be distinct buffers");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (p->opts.flags & MJK_FLAG_CHECK) {
        HIP_TRY(hipStreamSynchronize(s));
        if (int rc = check_density_host(p, D)) return rc;
    }
    const int64_t n2 = (int64_t)p->nbf * p->nbf;
    if (launch_fill(J, n2, 0.0, s) || launch_fill(K, n2, 0.0, s))
        return fail(MJK_ERR_HIP, "mjk_build_jk: fill launch failed");
    char *w = p->ws;
    if (p->timing && p->ev.size() != 2 * p->lists.size()) {
        for (auto e : p->ev) hipEventDestroy(e);
        p->ev.assign(2 * p->lists.size(), nullptr);
        for (auto &e : p->ev) HIP_TRY(hipEventCreate(&e));
    }
    p->timed_last = p->timing;
    for (size_t il = 0; il < p->lists.size(); ++il) {
        const WorkList &wl = p->lists[il];
        if (wl.nitems <= 0) continue;
        const BinPair &bp = p->bps[wl.bp];
        const Bin &X = p->bins[bp.X], &Y = p->bins[bp.Y];
        const int32_t *wk = (const int32_t *)(w + p->o_work) + wl.off;
        JKLaunch a{};
        a.pairs = (const ShellPairD *)(w + p->o_psort);
        a.prims = (const PrimPairD *)(w + p->o_prims);
        a.D = D;
        a.J = J;
        a.K = K;
        a.nbf = p->nbf;
        a.bra_begin = X.begin;
        a.nbra = X.count;
        a.ket_begin = Y.begin;
        a.same_bin = bp.X == bp.Y;
        a.ket_start = wk;
        a.ket_end = wk + X.count;
        a.chunk_prefix = wk + 2 * X.count;
        a.nitems = wl.nitems;
        a.chunk = kChunk;
        a.stage = (double *)(w + p->o_stage);
        a.nslot = p->nslot;
        const ClassEntry &ce = kClassTable[bp.qcls];
        if (p->timing) HIP_TRY(hipEventRecord(p->ev[2 * il], s));
        if ((wl.fp32 ? ce.jk32 : ce.jk)(a, s)) return fail(MJK_ERR_HIP, "mjk_build_jk: class launch failed");
        if (p->timing) HIP_TRY(hipEventRecord(p->ev[2 * il + 1], s));
    }
    if (launch_symmetrize(J, p->nbf, s) || launch_symmetrize(K, p->nbf, s))
        return fail(MJK_ERR_HIP, "mjk_build_jk: symmetrize launch failed");
    return MJK_OK;
}

int mjk_eri_class(mjk_plan *p, const int32_t *quartets, int64_t nq, double *out, int64_t out_len, void *stream)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_eri_class: plan is NULL");
    if (!p->bound) return fail(MJK_ERR_STATE, "mjk_eri_class: plan is not bound");
    if (nq < 0 || (nq > 0 && (!quartets || !out)))
        return fail(MJK_ERR_INVALID_ARG, "mjk_eri_class: bad quartet list");
    // canonicalize and group by quartet class
    std::vector<std::vector<EriItem>> groups(kNumQuartetClasses);
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
        groups[qc].push_back(it);
    }
    if (total != out_len)
        return fail(MJK_ERR_INVALID_ARG, "mjk_eri_class: out_len %lld, quartets need %lld", (long long)out_len,
                    (long long)total);
    if (nq == 0) return MJK_OK;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    char *w = p->ws;
    auto *stage = (EriItem *)(w + p->o_eri);
    for (int qc = 0; qc < kNumQuartetClasses; ++qc) {
        const auto &g = groups[qc];
        for (size_t i0 = 0; i0 < g.size(); i0 += kEriStage) {
            const int n = (int)std::min<size_t>(kEriStage, g.size() - i0);
            // stream order keeps this copy behind the previous launch that read the stage
            HIP_TRY(hipMemcpyAsync(stage, g.data() + i0, sizeof(EriItem) * n, hipMemcpyHostToDevice, s));
            EriLaunch a{(const ShellPairD *)(w + p->o_pnat), (const PrimPairD *)(w + p->o_prims), stage, n, out};
            if (kClassTable[qc].eri(a, s)) return fail(MJK_ERR_HIP, "mjk_eri_class: launch failed");
            HIP_TRY(hipStreamSynchronize(s));  // the host vector g is pageable and reused
        }
    }
    return MJK_OK;
}

int mjk_schwarz(mjk_plan *p, double *Qh)
{
    if (!p || !Qh) return fail(MJK_ERR_INVALID_ARG, "mjk_schwarz: NULL argument");
    if (!p->bound) return fail(MJK_ERR_STATE, "mjk_schwarz: plan is not bound");
    const int ns = p->nshell;
    for (int A = 0, k = 0; A < ns; ++A)
        for (int B = 0; B <= A; ++B, ++k) Qh[A * ns + B] = Qh[B * ns + A] = p->Q[k];
    return MJK_OK;
}

int mjk_plan_set_timing(mjk_plan *p, int enable)
{
    if (!p) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_set_timing: plan is NULL");
    p->timing = enable != 0;
    return MJK_OK;
}

int mjk_plan_timings(mjk_plan *p, mjk_class_timing *out, int32_t cap, int32_t *n)
{
    if (!p || !n || (cap > 0 && !out)) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_timings: NULL argument");
    if (!p->timed_last || p->ev.size() != 2 * p->lists.size())
        return fail(MJK_ERR_STATE, "mjk_plan_timings: the last build ran without timing");
    std::vector<mjk_class_timing> acc(kNumQuartetClasses);
    for (int q = 0; q < kNumQuartetClasses; ++q) {
        acc[q] = mjk_class_timing{};
        acc[q].la = kClassTable[q].la;
        acc[q].lb = kClassTable[q].lb;
        acc[q].lc = kClassTable[q].lc;
        acc[q].ld = kClassTable[q].ld;
    }
    for (size_t il = 0; il < p->lists.size(); ++il) {
        const auto &wl = p->lists[il];
        if (wl.nitems <= 0) continue;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev[2 * il], p->ev[2 * il + 1]));
        auto &t = acc[p->bps[wl.bp].qcls];
        t.nlaunch += 1;
        t.ms += ms;
        t.nquartet += wl.nq;
        t.nprim_quartet += wl.npq;
        t.flops += wl.cost;
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

int mjk_plan_stats_get(const mjk_plan *p, mjk_plan_stats *st)
{
    if (!p || !st) return fail(MJK_ERR_INVALID_ARG, "mjk_plan_stats_get: NULL argument");
    *st = p->stats;
    return MJK_OK;
}

}  // extern "C"
