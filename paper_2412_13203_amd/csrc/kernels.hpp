// kernels.hpp -- class-templated ERI kernels for gfx950 (wave64).
//
// Per primitive quartet (Eq. 2's summand) the device builds the geometry of
// the Obara-Saika recurrence, the Boys function F_m(T) for m <= L, the base
// integrals [00|00]^(m) = prefactor * F_m(T), and runs the generated vertical
// recurrence, accumulating [e0|f0] over the primitive quartets of the shell
// quartet (the contraction of Eq. 2).  The generated horizontal recurrence
// then gives the Cartesian block (ab|cd), which the J/K kernel digests at
// once into J and K (Section 7: the compute-bound ERIs fused with their
// memory-bound neighbour, reduced with atomics).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mjk_types.hpp"
#include "stage_guard.hpp"

namespace mjk {

template <typename T>
struct VrrGeom {
    T PA[3], WP[3], QC[3], WQ[3];
    T oo2p, oo2q, oo2pq, rho_p, rho_q;
};

template <int LA, int LB, int LC, int LD>
struct EriClass;

template <int LA, int LB, int LC, int LD>
struct EriSplit;

}  // namespace mjk

#include "gen/boys_table.inc"

namespace mjk {

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// The tables the kernels read (pairs, primitive pairs, work lists, segments,
// D) are not written while a kernel runs.  Loads through these constant
// (address space 4) views become scalar loads where the address is uniform
// and global loads elsewhere, instead of generic flat loads, which also tie
// up the LDS/scalar counters.  Never used for memory a kernel writes.
template <typename T>
using gptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> gview(const T *p)
{
    return (gptr<T>)p;
}

template <typename T>
__device__ __forceinline__ T ldg(const T *p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return *gview(p);
#else
    return *p;  // the host pass only parses device code
#endif
}

// ---------------------------------------------------------------------------
// Boys function F_m(T), m = 0..L (Section 2.2's analytic [00|00] needs it).
// T < TMAX: Taylor expansion of F_L and exp(-T) about the nearest grid point
// of a build-time table, then downward recursion
//     F_m = (2T F_{m+1} + exp(-T)) / (2m + 1).
// T >= TMAX: F_0 = sqrt(pi/T)/2 (erfc(sqrt T) < 1e-18 there) and the upward
// recursion F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T), stable for T >> m.
// ---------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ void boys_fm(double T, double *F)
{
    static_assert(L <= MJK_BOYS_LMAX, "Boys table too short for this class");
    constexpr int K = MJK_BOYS_KTAY;
    if (T < (double)MJK_BOYS_TMAX) {
        const int i = (int)(T * (double)MJK_BOYS_DT_INV + 0.5);
        const double md = (double)i * (1.0 / MJK_BOYS_DT_INV) - T;  // -(T - T0), |md| <= 1/32
        const double *row = mjk_boys_table + i * MJK_BOYS_NCOL;
        double f = row[L + K - 1];
        double e = 1.0;
#pragma unroll
        for (int k = K - 1; k >= 1; --k) {
            const double s = md * (1.0 / (double)k);
            f = row[L + k - 1] + f * s;
            e = 1.0 + e * s;
        }
        const double eT = row[MJK_BOYS_NCOL - 1] * e;
        F[L] = f;
        const double T2 = 2.0 * T;
#pragma unroll
        for (int m = L - 1; m >= 0; --m) F[m] = (T2 * F[m + 1] + eT) * (1.0 / (double)(2 * m + 1));
    } else {
        const double rT = 1.0 / T;
        const double eT = exp(-T);
        F[0] = 0.5 * sqrt(3.14159265358979323846 * rT);
        const double h = 0.5 * rT;
#pragma unroll
        for (int m = 0; m < L; ++m) F[m + 1] = ((double)(2 * m + 1) * F[m] - eT) * h;
    }
}

// Geometry of one primitive quartet, Obara-Saika notation:
// rho = pq/(p+q), W = (pP + qQ)/(p+q), WP = W - P = -q/(p+q) PQ,
// WQ = W - Q = p/(p+q) PQ, T = rho |PQ|^2, prefactor K_bra K_ket / sqrt(p+q).
__device__ __forceinline__ double prim_geom(const PrimPairD &b, const PrimPairD &k, VrrGeom<double> &g,
                                            double &T)
{
    const double PQx = b.P[0] - k.P[0], PQy = b.P[1] - k.P[1], PQz = b.P[2] - k.P[2];
    const double r = rsqrt(b.p + k.p);
    const double ipq = r * r;
    const double rho_p = k.p * ipq, rho_q = b.p * ipq;
    const double rho = b.p * rho_p;
    T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    g.PA[0] = b.PA[0];
    g.PA[1] = b.PA[1];
    g.PA[2] = b.PA[2];
    g.QC[0] = k.PA[0];
    g.QC[1] = k.PA[1];
    g.QC[2] = k.PA[2];
    g.WP[0] = -rho_p * PQx;
    g.WP[1] = -rho_p * PQy;
    g.WP[2] = -rho_p * PQz;
    g.WQ[0] = rho_q * PQx;
    g.WQ[1] = rho_q * PQy;
    g.WQ[2] = rho_q * PQz;
    g.oo2p = b.oo2p;
    g.oo2q = k.oo2p;
    g.oo2pq = 0.5 * ipq;
    g.rho_p = rho_p;
    g.rho_q = rho_q;
    return b.K * k.K * r;
}

__device__ __forceinline__ PrimPairD load_prim(const PrimPairD *__restrict__ p)
{
    return ldg(p);
}


// Primitive weights of the derivative integrals: none, 2 alpha (first bra
// centre), 2 beta (second bra centre), 2 gamma (first ket centre).
enum { WK_ONE = 0, WK_A = 1, WK_B = 2, WK_C = 3 };

// Loop over the primitive quartets of one shell quartet, ket primitives
// outer (each lane loads its own ket record once), bra primitives inner
// (wave-uniform records: scalar loads).  body(F, g) receives
// [00|00]^(m) = prefactor * F_m(T), m = 0..L, and the recurrence geometry;
// WK != WK_ONE also multiplies the prefactor by that primitive weight.
template <int L, int WK = WK_ONE, typename Body>
__device__ __forceinline__ void prim_loop(const ShellPairD &bra, const ShellPairD &ket,
                                          const PrimPairD *__restrict__ prims, bool active, Body &&body)
{
    const int nk = active ? ket.nprim : 0;
    for (int ik = 0; ik < nk; ++ik) {
        const PrimPairD kp = load_prim(prims + ket.prim_off + ik);
        for (int ib = 0; ib < bra.nprim; ++ib) {
            const PrimPairD bp = load_prim(prims + bra.prim_off + ib);
            VrrGeom<double> g;
            double T;
            double pref = prim_geom(bp, kp, g, T);
            if constexpr (WK == WK_A) pref *= 2.0 * bp.alpha;
            if constexpr (WK == WK_B) pref *= 2.0 * (bp.p - bp.alpha);
            if constexpr (WK == WK_C) pref *= 2.0 * kp.alpha;
            double F[L + 1];
            boys_fm<L>(T, F);
#pragma unroll
            for (int m = 0; m <= L; ++m) F[m] *= pref;
            body(F, g);
        }
    }
}

// Contracted [e0|f0] of one shell quartet: loop over its primitive quartets.
// Hand the recurrence its inputs in the accumulation type T: for T = float
// the geometry and Boys values (computed in FP64) are rounded to FP32 here.
template <typename T>
__device__ __forceinline__ void to_type(const VrrGeom<double> &g, VrrGeom<T> &h)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        h.PA[i] = (T)g.PA[i];
        h.WP[i] = (T)g.WP[i];
        h.QC[i] = (T)g.QC[i];
        h.WQ[i] = (T)g.WQ[i];
    }
    h.oo2p = (T)g.oo2p;
    h.oo2q = (T)g.oo2q;
    h.oo2pq = (T)g.oo2pq;
    h.rho_p = (T)g.rho_p;
    h.rho_q = (T)g.rho_q;
}

template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void contract_quartet(const ShellPairD &bra, const ShellPairD &ket,
                                                 const PrimPairD *__restrict__ prims, bool active, T *acc)
{
    using C = EriClass<LA, LB, LC, LD>;
    constexpr int L = LA + LB + LC + LD;
#pragma unroll
    for (int i = 0; i < C::NACC; ++i) acc[i] = T(0);
    prim_loop<L>(bra, ket, prims, active, [&](const double *F, const VrrGeom<double> &g) {
        if constexpr (sizeof(T) == sizeof(double)) {
            C::template vrr<double>(F, g, acc);
        } else {
            T Ft[L + 1];
#pragma unroll
            for (int m = 0; m <= L; ++m) Ft[m] = (T)F[m];
            VrrGeom<T> h;
            to_type(g, h);
            C::template vrr<T>(Ft, h, acc);
        }
    });
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Work items.  A launch covers the segments of one class (bin pairs of one or
// many molecules); item i belongs to the last segment with item_begin <= i,
// and inside it to the bra whose chunk range holds it.  All of this is
// wave-uniform (scalar loads).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_seg(const JKLaunch &a, int item)
{
    int lo = 0, hi = a.nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ldg(&a.segs[mid].item_begin) <= item)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void locate(const JKSeg &sg, int local, int &b, int &kbeg, int &kend)
{
    int lo = 0, hi = sg.nbra;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ldg(sg.chunk_prefix + mid) <= local)
            lo = mid;
        else
            hi = mid;
    }
    b = lo;
    kbeg = (local - ldg(sg.chunk_prefix + b)) * sg.chunk;
    kend = min(kbeg + sg.chunk, ldg(sg.ket_count + b));
}

// the kept run of bra b that holds its ket number k (uniform)
__device__ __forceinline__ int find_run(const JKSeg &sg, int b, int k)
{
    int lo = ldg(sg.run_begin + b), hi = ldg(sg.run_begin + b + 1);
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ldg(&sg.runs[mid].start) <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Kets of one round: ket numbers k0 + lane of the current bra.  `r` is the
// run holding k0 and `rend` one past the bra's last run (both uniform); r is
// advanced to the run holding k0 + 64.  Lane j looks at the start of run
// r + 1 + j; runs are never empty, so at most 63 of them start inside the
// round and a 6-step search over those starts finds each lane's run.
struct RoundKets {
    int pos;    // bin position of the lane's ket (meaningless past the bra's last ket)
    int last;   // last lane of the lane's run inside the round
    bool head;  // the lane is the first of its run inside the round
};

__device__ __forceinline__ RoundKets round_kets(const JKSeg &sg, int &r, int rend, int k0, int lane)
{
    const KetRun cur = ldg(sg.runs + r);
    const int rj = r + 1 + lane;
    KetRun nx{0, 0};
    if (rj < rend) nx = ldg(sg.runs + rj);
    const int dj = rj < rend ? nx.start - k0 : (1 << 30);  // lane at which run r + 1 + j starts (>= 1)
    int c = 0;  // runs after r that start at or before this lane
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const int t = __shfl(dj, c + step - 1, 64);
        if (t <= lane) c += step;
    }
    const int src = c > 0 ? c - 1 : 0;
    const int s1 = __shfl(nx.start, src, 64), p1 = __shfl(nx.pos, src, 64);
    const int nxt = __shfl(dj, c, 64);
    const int s = c > 0 ? s1 : cur.start, p = c > 0 ? p1 : cur.pos;
    RoundKets o;
    o.pos = p + (k0 + lane - s);
    o.last = min(nxt - 1, 63);
    o.head = lane == 0 || s == k0 + lane;
    r += __popcll(__ballot(dj <= 64));
    return o;
}

// sum of v over lanes [lane, last] (a segmented suffix sum; `last` is the
// last lane of the lane's run, so at a run's head lane this is the run total)
__device__ __forceinline__ double run_suffix_sum(double v, int lane, int last)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_down(v, d, 64);
        if (lane + d <= last) v += o;
    }
    return v;
}

// persistent blocks (one wave each) take items from the launch's counter;
// the item is wave-uniform and is kept in a scalar register, so that the
// segment and pair records decoded from it are scalar loads, as they are for
// a block-indexed item
__device__ __forceinline__ int next_item(const JKLaunch &a, int lane)
{
    int v = 0;
    if (lane == 0) v = (int)atomicAdd(a.queue, 1u);
    return __builtin_amdgcn_readfirstlane(__shfl(v, 0, 64));
}

// per-molecule wall-clock stamps: first item start, last item end
__device__ __forceinline__ void stamp(const JKLaunch &a, int mol, int lane, bool end)
{
    if (a.stamps != nullptr && lane == 0) {
        const unsigned long long t = (unsigned long long)wall_clock64();
        if (end)
            atomicMax(a.stamps + 2 * mol + 1, t);
        else
            atomicMin(a.stamps + 2 * mol, t);
    }
}

// ---------------------------------------------------------------------------
// Fused J/K: one wave = one bra pair (uniform) x up to 64 ket pairs per
// round (one per lane), `chunk` kets per item; persistent waves pop items.  Digestion of (ab|cd) with the 8-fold symmetry of a
// unique quartet, weight w = 1/(s_AB s_CD s_ABCD):
//   Jt_ab += 2w D_cd   Jt_cd += 2w D_ab
//   Kt_ac += w D_bd    Kt_ad += w D_bc    Kt_bc += w D_ad    Kt_bd += w D_ac
// J = Jt + Jt^T and K = Kt + Kt^T afterwards (k_symmetrize).  Jt_ab is
// bra-uniform, so it is reduced across the wave before its atomic; Kt_ac and
// Kt_bc depend on the ket only through C, so they are summed over the lanes
// of one run (same C) and added once per run.
// ---------------------------------------------------------------------------
template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void jk_lane_item(const JKLaunch &a, int item)
{
    using C = EriClass<LA, LB, LC, LD>;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    const int lane = threadIdx.x;
    const JKSeg sg = ldg(a.segs + find_seg(a, item));
    int b, kbeg, kend;
    locate(sg, item - sg.item_begin, b, kbeg, kend);
    stamp(a, sg.mol, lane, false);
    const int bra_pos = sg.bra_begin + b;
    const ShellPairD bra = ldg(sg.pairs + bra_pos);
    const int N = sg.nbf;
    const gptr<double> __restrict__ D = gview(a.D + sg.mat_off);
    double *__restrict__ Jm = a.J + sg.mat_off;
    double *__restrict__ Km = a.K + sg.mat_off;
    int run = find_run(sg, b, kbeg);
    const int run_end = ldg(sg.run_begin + b + 1);

    double Dab[NA * NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) Dab[i * NB + j] = D[(size_t)(bra.ao_a + i) * N + bra.ao_b + j];
    double jab[NA * NB];
#pragma unroll
    for (int i = 0; i < NA * NB; ++i) jab[i] = 0.0;

    for (int k0 = kbeg; k0 < kend; k0 += 64) {
        const bool active = k0 + lane < kend;
        const RoundKets rk = round_kets(sg, run, run_end, k0, lane);
        const int pos0 = __builtin_amdgcn_readfirstlane(__shfl(rk.pos, 0, 64));
        const int ket_pos = sg.ket_begin + (active ? rk.pos : pos0);
        const ShellPairD ket = ldg(sg.pairs + ket_pos);
        T acc[C::NACC];
        contract_quartet<LA, LB, LC, LD, T>(bra, ket, sg.prims, active, acc);
        double eri[C::NOUT];
        if constexpr (sizeof(T) == sizeof(double)) {
            C::template hrr<double>(acc, bra.AB, ket.AB, eri);
        } else {
            // FP32 recurrence and contraction; the horizontal recurrence (whose
            // AB, CD factors amplify rounding) runs on the widened values
            double acc64[C::NACC];
#pragma unroll
            for (int i = 0; i < C::NACC; ++i) acc64[i] = (double)acc[i];
            C::template hrr<double>(acc64, bra.AB, ket.AB, eri);
        }

        double s = 1.0;
        if (bra.same) s *= 2.0;
        if (ket.same) s *= 2.0;
        if (sg.same_bin && ket_pos == bra_pos) s *= 2.0;
        const double w = active ? 1.0 / s : 0.0;

        double Dcd[NC * ND];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int d = 0; d < ND; ++d) Dcd[c * ND + d] = D[(size_t)(ket.ao_a + c) * N + ket.ao_b + d];
        // Jt_ab (wave-reduced later) and Jt_cd
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) {
            double t = 0.0;
#pragma unroll
            for (int cd = 0; cd < NC * ND; ++cd) t += eri[ab * NC * ND + cd] * Dcd[cd];
            jab[ab] += 2.0 * w * t;
        }
        // Kt_ac += w sum_{b,d} (ab|cd) D_bd and Kt_bc += w sum_{a,d} (ab|cd) D_ad,
        // summed over the run before the atomic (all lanes take part)
        const bool flush = active && rk.head;
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double t = 0.0;
#pragma unroll
                for (int jb = 0; jb < NB; ++jb)
#pragma unroll
                    for (int d = 0; d < ND; ++d)
                        t += eri[((ia * NB + jb) * NC + c) * ND + d] * D[(size_t)(bra.ao_b + jb) * N + ket.ao_b + d];
                t = run_suffix_sum(w * t, lane, rk.last);
                if (flush) atomicAdd(Km + (size_t)(bra.ao_a + ia) * N + ket.ao_a + c, t);
            }
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double t = 0.0;
#pragma unroll
                for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                    for (int d = 0; d < ND; ++d)
                        t += eri[((ia * NB + jb) * NC + c) * ND + d] * D[(size_t)(bra.ao_a + ia) * N + ket.ao_b + d];
                t = run_suffix_sum(w * t, lane, rk.last);
                if (flush) atomicAdd(Km + (size_t)(bra.ao_b + jb) * N + ket.ao_a + c, t);
            }
        if (active) {
#pragma unroll
            for (int cd = 0; cd < NC * ND; ++cd) {
                double t = 0.0;
#pragma unroll
                for (int ab = 0; ab < NA * NB; ++ab) t += eri[ab * NC * ND + cd] * Dab[ab];
                const int c = cd / ND, d = cd % ND;
                atomicAdd(Jm + (size_t)(ket.ao_a + c) * N + ket.ao_b + d, 2.0 * w * t);
            }
            // Kt_ad += w sum_{b,c} (ab|cd) D_bc ; Kt_bd += w sum_{a,c} (ab|cd) D_ac
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    double t = 0.0;
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            t += eri[((ia * NB + jb) * NC + c) * ND + d] *
                                 D[(size_t)(bra.ao_b + jb) * N + ket.ao_a + c];
                    atomicAdd(Km + (size_t)(bra.ao_a + ia) * N + ket.ao_b + d, w * t);
                }
#pragma unroll
            for (int jb = 0; jb < NB; ++jb)
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    double t = 0.0;
#pragma unroll
                    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            t += eri[((ia * NB + jb) * NC + c) * ND + d] *
                                 D[(size_t)(bra.ao_a + ia) * N + ket.ao_a + c];
                    atomicAdd(Km + (size_t)(bra.ao_b + jb) * N + ket.ao_b + d, w * t);
                }
        }
    }
#pragma unroll
    for (int ab = 0; ab < NA * NB; ++ab) {
        const double t = wave_sum(jab[ab]);
        if (lane == 0) atomicAdd(Jm + (size_t)(bra.ao_a + ab / NB) * N + bra.ao_b + ab % NB, t);
    }
    stamp(a, sg.mol, lane, true);
}

// One block per item, or (lane_persistent) persistent waves that take items
// from the launch's counter until none are left (the launch's grid is then
// the occupancy bound, cut to the items).
template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void jk_lane_body(const JKLaunch &a)
{
    if (!a.lane_persistent) {
        jk_lane_item<LA, LB, LC, LD, T>(a, blockIdx.x);
        return;
    }
    const int lane = threadIdx.x;
    for (;;) {
        const int item = next_item(a, lane);
        if (item >= a.nitems) break;
        jk_lane_item<LA, LB, LC, LD, T>(a, item);
    }
}

// Resident waves per SIMD asked of the compiler for a few per-lane classes
// whose register count sits just above an occupancy step (0: no request).
// Measured per class: (dp|ps) 264 VGPRs -> 256, 1 -> 2 waves, 7.4 -> 5.7 ms;
// (ds|pp) 280 -> 256, 5.6 -> 5.1 ms; (ps|ps) 130 -> 128, 2.31 -> 2.20 ms;
// (pp|ps) 191 -> 168, 1.89 -> 1.79 ms.  The same request slowed (ds|ps) and
// (pp|ss), whose reduced budgets spill.
template <int LA, int LB, int LC, int LD>
constexpr int jk_waves()
{
    return (LA == 2 && LB == 1 && LC == 1 && LD == 0)   ? 2
           : (LA == 2 && LB == 0 && LC == 1 && LD == 1) ? 2
           : (LA == 1 && LB == 0 && LC == 1 && LD == 0) ? 4
           : (LA == 1 && LB == 1 && LC == 1 && LD == 0) ? 3
                                                        : 0;
}

template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_jk(JKLaunch a)
{
    jk_lane_body<LA, LB, LC, LD, T>(a);
}

template <int LA, int LB, int LC, int LD, typename T, int W>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W))) void k_jk_occ(JKLaunch a)
{
    jk_lane_body<LA, LB, LC, LD, T>(a);
}

// ---------------------------------------------------------------------------
// Explicit ERI blocks: one requested quartet per lane, canonical class order,
// written back in the caller's shell order.  T = float: FP32 recurrence and
// contraction, HRR on the widened values (as in the J/K path).
// ---------------------------------------------------------------------------
template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_eri(EriLaunch a)
{
    using C = EriClass<LA, LB, LC, LD>;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= a.n) return;
    const EriItem it = a.items[t];
    const ShellPairD bra = a.pairs[it.bra];
    const ShellPairD ket = a.pairs[it.ket];
    T acc[C::NACC];
    contract_quartet<LA, LB, LC, LD, T>(bra, ket, a.prims, true, acc);
    double eri[C::NOUT];
    if constexpr (sizeof(T) == sizeof(double)) {
        C::template hrr<double>(acc, bra.AB, ket.AB, eri);
    } else {
        double acc64[C::NACC];
#pragma unroll
        for (int i = 0; i < C::NACC; ++i) acc64[i] = (double)acc[i];
        C::template hrr<double>(acc64, bra.AB, ket.AB, eri);
    }
    const bool sab = it.flags & 1, scd = it.flags & 2, sbk = it.flags & 4;
    double *out = a.out + it.out_off;
    for (int i = 0; i < NA; ++i)
        for (int j = 0; j < NB; ++j)
            for (int k = 0; k < NC; ++k)
                for (int l = 0; l < ND; ++l) {
                    int x1, x2, x3, x4;
                    if (!sbk) {
                        x1 = sab ? j : i;
                        x2 = sab ? i : j;
                        x3 = scd ? l : k;
                        x4 = scd ? k : l;
                    } else {
                        x1 = sab ? l : k;
                        x2 = sab ? k : l;
                        x3 = scd ? j : i;
                        x4 = scd ? i : j;
                    }
                    out[((size_t)(x1 * it.n2 + x2) * it.n3 + x3) * it.n4 + x4] =
                        eri[((i * NB + j) * NC + k) * ND + l];
                }
}

// ---------------------------------------------------------------------------
// Schwarz factors: Q_AB = sqrt(max_{a,b} (ab|ab)), one pair per lane.
// ---------------------------------------------------------------------------
template <int LA, int LB>
__global__ __launch_bounds__(64) void k_schwarz(SchwarzLaunch a)
{
    using C = EriClass<LA, LB, LA, LB>;
    constexpr int NA = ncart(LA), NB = ncart(LB);
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= a.n) return;
    const int pi = a.idx[t];
    const ShellPairD pr = a.pairs[pi];
    double acc[C::NACC];
    contract_quartet<LA, LB, LA, LB, double>(pr, pr, a.prims, true, acc);
    double eri[C::NOUT];
    C::template hrr<double>(acc, pr.AB, pr.AB, eri);
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < NA * NB; ++i) mx = fmax(mx, eri[i * NA * NB + i]);
    a.Q[pi] = sqrt(mx);
}

// ---------------------------------------------------------------------------
// Fused J/K for classes whose [e0|f0] accumulators do not fit one lane's
// registers.  Same work items as k_jk (one bra pair x up to 64 kets), but
//   phase 1: each lane runs the vertical recurrence in NPASS passes over its
//            quartet's primitive quartets; a pass keeps only its subset of
//            accumulators in registers and writes them to a per-slot staging
//            buffer in global memory, quartet-major with the targets in pass
//            order ([lane][pass, j]), through a 16-target LDS transpose so that
//            the stores are coalesced;
//   phase 2: the wave takes the item's quartets one at a time: [e0|f0] read
//            contiguously and scattered into LDS in target order, bra HRR one
//            ket column per lane, ket HRR one (ab) row per lane, then the six
//            digestion contractions one output element per lane, with the
//            bra-uniform Jt_ab kept per lane across the item.
// (The gradient's split passes keep the [target][lane] layout: their HRR reads
// the slot directly.)
// Blocks are persistent (grid = staging slots) and stride over the items.
// ---------------------------------------------------------------------------
// first staging position of pass P (positions are in pass order)
template <int LA, int LB, int LC, int LD, int P>
__device__ constexpr int split_off()
{
    if constexpr (P == 0)
        return 0;
    else
        return split_off<LA, LB, LC, LD, P - 1>() + EriSplit<LA, LB, LC, LD>::template npass_acc<P - 1>();
}

// target index of staging position s (pass order -> target order)
template <int LA, int LB, int LC, int LD, int P = 0>
__device__ __forceinline__ int split_target(int s)
{
    using S = EriSplit<LA, LB, LC, LD>;
    if constexpr (P >= S::NPASS) {
        return -1;
    } else {
        constexpr int o = split_off<LA, LB, LC, LD, P>(), n = S::template npass_acc<P>();
        if (s < o + n) return S::template gmap<P>(s - o);
        return split_target<LA, LB, LC, LD, P + 1>(s);
    }
}

// QMAJOR = false: the slot is [target][lane] (gradient); true: [lane][position]
// written through the wave's 16 x 65 LDS transpose buffer s_tr (J/K).
template <int LA, int LB, int LC, int LD, int P, typename T, int WK = WK_ONE, bool QMAJOR = false>
__device__ __forceinline__ void split_pass(const ShellPairD &bra, const ShellPairD &ket,
                                           const PrimPairD *__restrict__ prims, bool active,
                                           double *__restrict__ stage, int lane, double *s_tr = nullptr)
{
    using S = EriSplit<LA, LB, LC, LD>;
    constexpr int L = LA + LB + LC + LD;
    constexpr int NP = S::template npass_acc<P>();
    T acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = T(0);
    prim_loop<L, WK>(bra, ket, prims, active, [&](const double *F, const VrrGeom<double> &g) {
        if constexpr (sizeof(T) == sizeof(double)) {
            S::template vrr<P, double>(F, g, acc);
        } else {
            T Ft[L + 1];
#pragma unroll
            for (int m = 0; m <= L; ++m) Ft[m] = (T)F[m];
            VrrGeom<T> h;
            to_type(g, h);
            S::template vrr<P, T>(Ft, h, acc);
        }
    });
    if constexpr (QMAJOR) {
        // 16 positions at a time: lanes write their values to LDS, then each
        // store instruction writes 16 consecutive positions of 4 quartets
        // (lane-dependent offsets are made opaque, as below, so that the
        // compiler does not keep one address per store live across the item
        // loop)
        constexpr int O = split_off<LA, LB, LC, LD, P>();
        const int jj = lane & 15;
        int qo = (lane >> 4) * S::NACC + O + jj, to = jj * 65 + (lane >> 4), lo = lane;
        __asm__ volatile("" : "+v"(qo), "+v"(to), "+v"(lo));
        double *sq = stage + qo;
        const double *tr = s_tr + to;
        double *tw = s_tr + lo;
#pragma unroll
        for (int c0 = 0; c0 < NP; c0 += 16) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (c0 + j < NP) tw[j * 65] = (double)acc[c0 + j];
            __syncthreads();
            if (c0 + jj < NP) {
#pragma unroll
                for (int r = 0; r < 16; ++r) sq[4 * r * S::NACC + c0] = tr[4 * r];
            }
            __syncthreads();
        }
    } else {
        // The lane offset is made opaque here so that the compiler cannot hoist
        // one 64-bit store address per target out of the item loop (that many
        // live addresses would be spilled to scratch).
        int off = lane;
        __asm__ volatile("" : "+v"(off));
        double *sl = stage + off;
#pragma unroll
        for (int j = 0; j < NP; ++j) sl[S::template gmap<P>(j) * 64] = (double)acc[j];
    }
}

template <int LA, int LB, int LC, int LD, int P, typename T, int WK = WK_ONE, bool QMAJOR = false>
__device__ __forceinline__ void split_passes(const ShellPairD &bra, const ShellPairD &ket,
                                             const PrimPairD *__restrict__ prims, bool active,
                                             double *__restrict__ stage, int lane, double *s_tr = nullptr)
{
    if constexpr (P < EriSplit<LA, LB, LC, LD>::NPASS) {
        split_pass<LA, LB, LC, LD, P, T, WK, QMAJOR>(bra, ket, prims, active, stage, lane, s_tr);
        split_passes<LA, LB, LC, LD, P + 1, T, WK, QMAJOR>(bra, ket, prims, active, stage, lane, s_tr);
    }
}

// T = float: the passes run the recurrence and the contraction in FP32 and
// stage the contracted values as FP64; HRR and digestion are FP64.
template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void jk_split_body(const JKLaunch &a)
{
    using S = EriSplit<LA, LB, LC, LD>;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NAB = NA * NB, NCD = NC * ND, NF = S::NF, NACC = S::NACC;
    constexpr int NBUF = NACC > NAB * NCD ? NACC : NAB * NCD;
    // density blocks of one quartet: D_cd, D_ac, D_ad, D_bc, D_bd back to back
    constexpr int OAC = NCD, OAD = OAC + NA * NC, OBC = OAD + NA * ND, OBD = OBC + NB * NC, NDQ = OBD + NB * ND;
    constexpr int KS = (NACC + 63) / 64, KD = (NDQ + 63) / 64;
    constexpr int KS_PRE = KS <= 16 ? KS : 0;  // staged values prefetched per lane
    constexpr int KAB = (NAB + 63) / 64;        // bra elements per lane (2 for an (ff| bra)
    constexpr int KAC = (NA * NC + 63) / 64, KBC = (NB * NC + 63) / 64;
    __shared__ double s_buf[NBUF];     // [e][f], then (ab|cd) as [ab][cd]
    __shared__ double s_abf[NAB * NF]; // (ab|f] as [ab][f]
    __shared__ double s_Dab[NAB], s_Dq[NDQ];
    __shared__ double s_CD[64][3];
    __shared__ double s_w[64];
    __shared__ int s_ao[64][2];
    __shared__ double s_tr[16 * 65];
    double *const s_Dcd = s_Dq, *const s_Dac = s_Dq + OAC, *const s_Dad = s_Dq + OAD, *const s_Dbc = s_Dq + OBC,
                  *const s_Dbd = s_Dq + OBD;
    static_assert(split_off<LA, LB, LC, LD, S::NPASS>() == NACC, "passes must partition the targets");
    const int lane = threadIdx.x;
    double *stage = a.stage + (size_t)blockIdx.x * NACC * 64;
    int tpos[KS_PRE > 0 ? KS_PRE : 1];  // target of staging position lane + 64 k
#pragma unroll
    for (int k = 0; k < KS_PRE; ++k)
        tpos[k] = lane + 64 * k < NACC ? split_target<LA, LB, LC, LD>(lane + 64 * k) : 0;

    for (;;) {
        const int item = next_item(a, lane);
        if (item >= a.nitems) break;
        const JKSeg sg = ldg(a.segs + find_seg(a, item));
        int b, kbeg, kend;
        locate(sg, item - sg.item_begin, b, kbeg, kend);
        stamp(a, sg.mol, lane, false);
        const int bra_pos = sg.bra_begin + b;
        const ShellPairD bra = ldg(sg.pairs + bra_pos);
        const int N = sg.nbf;
        const gptr<double> __restrict__ D = gview(a.D + sg.mat_off);
        double *__restrict__ Jm = a.J + sg.mat_off;
        double *__restrict__ Km = a.K + sg.mat_off;
        for (int t = lane; t < NAB; t += 64) s_Dab[t] = D[(size_t)(bra.ao_a + t / NB) * N + bra.ao_b + t % NB];
        double jab[KAB];  // Jt_ab for ab = lane + 64 k (< NAB), summed over the item
#pragma unroll
        for (int k = 0; k < KAB; ++k) jab[k] = 0.0;
        // Kt_ac and Kt_bc of the current C (element lane + 64 k), summed over
        // consecutive quartets of one run and added when C changes
        double kac[KAC], kbc[KBC];
#pragma unroll
        for (int k = 0; k < KAC; ++k) kac[k] = 0.0;
#pragma unroll
        for (int k = 0; k < KBC; ++k) kbc[k] = 0.0;
        int cur_c = -1;
        auto flush_c = [&]() {
#pragma unroll
            for (int k = 0; k < KAC; ++k) {
                const int t = lane + 64 * k;
                if (t < NA * NC) atomicAdd(Km + (size_t)(bra.ao_a + t / NC) * N + cur_c + t % NC, kac[k]);
                kac[k] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < KBC; ++k) {
                const int t = lane + 64 * k;
                if (t < NB * NC) atomicAdd(Km + (size_t)(bra.ao_b + t / NC) * N + cur_c + t % NC, kbc[k]);
                kbc[k] = 0.0;
            }
        };
        int run = find_run(sg, b, kbeg);
        const int run_end = ldg(sg.run_begin + b + 1);

        for (int k0 = kbeg; k0 < kend; k0 += 64) {
            // phase 1: one quartet per lane, passes into the staging slot
            const int nact = min(kend - k0, 64);
            const bool active = lane < nact;
            const RoundKets rk = round_kets(sg, run, run_end, k0, lane);
            const int pos0 = __builtin_amdgcn_readfirstlane(__shfl(rk.pos, 0, 64));
            const int ket_pos = sg.ket_begin + (active ? rk.pos : pos0);
            const ShellPairD ket = ldg(sg.pairs + ket_pos);
            split_passes<LA, LB, LC, LD, 0, T, WK_ONE, true>(bra, ket, sg.prims, active, stage, lane, s_tr);
            {
                double s = 1.0;
                if (bra.same) s *= 2.0;
                if (ket.same) s *= 2.0;
                if (sg.same_bin && ket_pos == bra_pos) s *= 2.0;
                s_w[lane] = active ? 1.0 / s : 0.0;
                s_CD[lane][0] = ket.AB[0];
                s_CD[lane][1] = ket.AB[1];
                s_CD[lane][2] = ket.AB[2];
                s_ao[lane][0] = ket.ao_a;
                s_ao[lane][1] = ket.ao_b;
            }
            __syncthreads();

            // phase 2: the wave works through this round's quartets.  The
            // staged [e0|f0] and the density blocks of quartet q + 1 are
            // loaded into registers while quartet q is digested (the staged
            // values only up to KS_PRE per lane; larger classes copy them
            // from the slot when their quartet starts).
            double pst[KS_PRE > 0 ? KS_PRE : 1], pdq[KD];
            auto fetch = [&](int q) {
                const int ao_c = s_ao[q][0], ao_d = s_ao[q][1];
#pragma unroll
                for (int k = 0; k < KS_PRE; ++k) {
                    const int t = lane + 64 * k;
                    pst[k] = t < NACC ? stage[(size_t)q * NACC + t] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < KD; ++k) {
                    const int t = lane + 64 * k;
                    size_t at = 0;
                    if (t < OAC)
                        at = (size_t)(ao_c + t / ND) * N + ao_d + t % ND;
                    else if (t < OAD)
                        at = (size_t)(bra.ao_a + (t - OAC) / NC) * N + ao_c + (t - OAC) % NC;
                    else if (t < OBC)
                        at = (size_t)(bra.ao_a + (t - OAD) / ND) * N + ao_d + (t - OAD) % ND;
                    else if (t < OBD)
                        at = (size_t)(bra.ao_b + (t - OBC) / NC) * N + ao_c + (t - OBC) % NC;
                    else if (t < NDQ)
                        at = (size_t)(bra.ao_b + (t - OBD) / ND) * N + ao_d + (t - OBD) % ND;
                    pdq[k] = t < NDQ ? D[at] : 0.0;
                }
            };
            fetch(0);
            for (int q = 0; q < nact; ++q) {
                const int ao_c = s_ao[q][0], ao_d = s_ao[q][1];
                if (ao_c != cur_c) {
                    if (cur_c >= 0) flush_c();
                    cur_c = ao_c;
                }
                if constexpr (KS_PRE == KS) {
#pragma unroll
                    for (int k = 0; k < KS; ++k)
                        if (lane + 64 * k < NACC) s_buf[tpos[k]] = pst[k];
                } else {
                    for (int t = lane; t < NACC; t += 64) s_buf[split_target<LA, LB, LC, LD>(t)] =
                        stage[(size_t)q * NACC + t];
                }
#pragma unroll
                for (int k = 0; k < KD; ++k)
                    if (lane + 64 * k < NDQ) s_Dq[lane + 64 * k] = pdq[k];
                __syncthreads();
                if (q + 1 < nact) fetch(q + 1);
                for (int f = lane; f < NF; f += 64) S::template hrr_bra_col<1, double>(s_buf, f, bra.AB, s_abf);
                __syncthreads();
                const double CD[3] = {s_CD[q][0], s_CD[q][1], s_CD[q][2]};
                const double w = s_w[q];
#pragma unroll
                for (int k = 0; k < KAB; ++k) {
                    const int r = lane + 64 * k;
                    if (r < NAB) {
                        double row[NCD];
                        S::template hrr_ket_row<double>(s_abf + r * NF, CD, row);
                        double t = 0.0;
#pragma unroll
                        for (int cd = 0; cd < NCD; ++cd) {
                            s_buf[r * NCD + cd] = row[cd];
                            t += row[cd] * s_Dcd[cd];
                        }
                        jab[k] += 2.0 * w * t;
                    }
                }
                __syncthreads();
                // Jt_cd += 2w sum_ab (ab|cd) D_ab
                for (int t = lane; t < NCD; t += 64) {
                    double v = 0.0;
#pragma unroll
                    for (int ab = 0; ab < NAB; ++ab) v += s_buf[ab * NCD + t] * s_Dab[ab];
                    atomicAdd(Jm + (size_t)(ao_c + t / ND) * N + ao_d + t % ND, 2.0 * w * v);
                }
                // Kt_ac += w sum_{b,d} (ab|cd) D_bd (held until C changes)
#pragma unroll
                for (int k = 0; k < KAC; ++k) {
                    const int t = lane + 64 * k;
                    if (t < NA * NC) {
                        const int ia = t / NC, c = t % NC;
                        double v = 0.0;
#pragma unroll
                        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
                            for (int d = 0; d < ND; ++d)
                                v += s_buf[(ia * NB + jb) * NCD + c * ND + d] * s_Dbd[jb * ND + d];
                        kac[k] += w * v;
                    }
                }
                // Kt_ad += w sum_{b,c} (ab|cd) D_bc
                for (int t = lane; t < NA * ND; t += 64) {
                    const int ia = t / ND, d = t % ND;
                    double v = 0.0;
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            v += s_buf[(ia * NB + jb) * NCD + c * ND + d] * s_Dbc[jb * NC + c];
                    atomicAdd(Km + (size_t)(bra.ao_a + ia) * N + ao_d + d, w * v);
                }
                // Kt_bc += w sum_{a,d} (ab|cd) D_ad (held until C changes)
#pragma unroll
                for (int k = 0; k < KBC; ++k) {
                    const int t = lane + 64 * k;
                    if (t < NB * NC) {
                        const int jb = t / NC, c = t % NC;
                        double v = 0.0;
#pragma unroll
                        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                            for (int d = 0; d < ND; ++d)
                                v += s_buf[(ia * NB + jb) * NCD + c * ND + d] * s_Dad[ia * ND + d];
                        kbc[k] += w * v;
                    }
                }
                // Kt_bd += w sum_{a,c} (ab|cd) D_ac
                for (int t = lane; t < NB * ND; t += 64) {
                    const int jb = t / ND, d = t % ND;
                    double v = 0.0;
#pragma unroll
                    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            v += s_buf[(ia * NB + jb) * NCD + c * ND + d] * s_Dac[ia * NC + c];
                    atomicAdd(Km + (size_t)(bra.ao_b + jb) * N + ao_d + d, w * v);
                }
                __syncthreads();
            }
        }
        if (cur_c >= 0) flush_c();
#pragma unroll
        for (int k = 0; k < KAB; ++k) {
            const int t = lane + 64 * k;
            if (t < NAB) atomicAdd(Jm + (size_t)(bra.ao_a + t / NB) * N + bra.ao_b + t % NB, jab[k]);
        }
        stamp(a, sg.mol, lane, true);
        __syncthreads();
    }
}

// Phase 1 of the split eri kernel, one code path for both forms (the pass
// code is instantiated once): each lane sums the primitive quartets
// ip = pstart, pstart + pstep, ... of its quartet (bra, ket).  reduce = false:
// one quartet per lane, its sums stored quartet-major as in the J/K kernel.
// reduce = true: the wave's lanes share one quartet (pstart = lane,
// pstep = 64, the contraction of Eq. 2 spread over the wave) and their sums
// are added through the 16 x 65 LDS buffer s_tr, 16 accumulators at a time,
// each by one lane in a fixed order, and stored as quartet 0 of the slot.
template <int LA, int LB, int LC, int LD, int P, typename T>
__device__ __forceinline__ void eri_passes(const ShellPairD &bra, const ShellPairD &ket,
                                           const PrimPairD *__restrict__ prims, bool active,
                                           double *__restrict__ stage, int lane, double *__restrict__ s_tr,
                                           int pstart, int pstep, bool reduce)
{
    using S = EriSplit<LA, LB, LC, LD>;
    if constexpr (P < S::NPASS) {
        constexpr int L = LA + LB + LC + LD;
        constexpr int NP = S::template npass_acc<P>(), O = split_off<LA, LB, LC, LD, P>();
        T acc[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) acc[i] = T(0);
        const int nb = bra.nprim, npq = active ? nb * ket.nprim : 0;
        for (int ip = pstart; ip < npq; ip += pstep) {
            const PrimPairD kp = load_prim(prims + ket.prim_off + ip / nb);
            const PrimPairD bp = load_prim(prims + bra.prim_off + ip % nb);
            VrrGeom<double> g;
            double Tb;
            const double pref = prim_geom(bp, kp, g, Tb);
            double F[L + 1];
            boys_fm<L>(Tb, F);
#pragma unroll
            for (int m = 0; m <= L; ++m) F[m] *= pref;
            if constexpr (sizeof(T) == sizeof(double)) {
                S::template vrr<P, double>(F, g, acc);
            } else {
                T Ft[L + 1];
#pragma unroll
                for (int m = 0; m <= L; ++m) Ft[m] = (T)F[m];
                VrrGeom<T> h;
                to_type(g, h);
                S::template vrr<P, T>(Ft, h, acc);
            }
        }
        if (reduce) {
#pragma unroll
            for (int c0 = 0; c0 < NP; c0 += 16) {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (c0 + j < NP) s_tr[j * 65 + lane] = (double)acc[c0 + j];
                __syncthreads();
                if (lane < 16 && c0 + lane < NP) {
                    double v = 0.0;
                    for (int l = 0; l < 64; ++l) v += s_tr[lane * 65 + l];
                    stage[O + c0 + lane] = v;
                }
                __syncthreads();
            }
        } else {
            // quartet-major store through the transpose, as split_pass does
            const int jj = lane & 15;
            int qo = (lane >> 4) * S::NACC + O + jj, to = jj * 65 + (lane >> 4), lo = lane;
            __asm__ volatile("" : "+v"(qo), "+v"(to), "+v"(lo));
            double *sq = stage + qo;
            const double *tr = s_tr + to;
            double *tw = s_tr + lo;
#pragma unroll
            for (int c0 = 0; c0 < NP; c0 += 16) {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (c0 + j < NP) tw[j * 65] = (double)acc[c0 + j];
                __syncthreads();
                if (c0 + jj < NP) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) sq[4 * r * S::NACC + c0] = tr[4 * r];
                }
                __syncthreads();
            }
        }
        eri_passes<LA, LB, LC, LD, P + 1, T>(bra, ket, prims, active, stage, lane, s_tr, pstart, pstep, reduce);
    }
}

// ---------------------------------------------------------------------------
// Explicit ERI blocks (and Schwarz factors) of classes split into recurrence
// passes: persistent blocks take 64 requested quartets at a time; phase 1 as
// in the split J/K kernel (one quartet per lane, passes into the block's
// staging slot), or, with `deconstruct`, one quartet at a time with its
// primitive quartets spread over the lanes; phase 2 one quartet at a time: bra HRR one ket column per
// lane, ket HRR one (ab) row per lane, then the block written in the
// caller's shell order, or, in Schwarz mode (a.Q set, items (pair, pair)),
// Q = sqrt(max_{a,b} (ab|ab)) written for the pair.
// ---------------------------------------------------------------------------
template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_eri_split(EriLaunch a)
{
    using S = EriSplit<LA, LB, LC, LD>;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NAB = NA * NB, NCD = NC * ND, NF = S::NF, NACC = S::NACC;
    constexpr int NBUF = NACC > NAB * NCD ? NACC : NAB * NCD;
    __shared__ double s_buf[NBUF];     // [e][f], then (ab|cd) as [ab][cd]
    __shared__ double s_abf[NAB * NF]; // (ab|f] as [ab][f]
    __shared__ double s_tr[16 * 65];
    static_assert(split_off<LA, LB, LC, LD, S::NPASS>() == NACC, "passes must partition the targets");
    const int lane = threadIdx.x;
    double *stage = a.stage + (size_t)blockIdx.x * NACC * 64;
    const bool decon = a.deconstruct != 0;
    const int gsize = decon ? 1 : 64;  // quartets per group
    const int ngroup = (a.n + gsize - 1) / gsize;
    for (int grp = blockIdx.x; grp < ngroup; grp += gridDim.x) {
        const int t0 = grp * gsize;
        const int nact = min(a.n - t0, gsize);
        {
            const bool active = decon || lane < nact;
            const EriItem it = a.items[t0 + (decon || !active ? 0 : lane)];
            eri_passes<LA, LB, LC, LD, 0, T>(a.pairs[it.bra], a.pairs[it.ket], a.prims, active, stage, lane, s_tr,
                                            decon ? lane : 0, decon ? 64 : 1, decon);
        }
        __syncthreads();
        for (int q = 0; q < nact; ++q) {
            const EriItem iq = a.items[t0 + q];
            const ShellPairD bq = a.pairs[iq.bra];
            const ShellPairD kq = a.pairs[iq.ket];
            for (int t = lane; t < NACC; t += 64) s_buf[split_target<LA, LB, LC, LD>(t)] = stage[(size_t)q * NACC + t];
            __syncthreads();
            for (int f = lane; f < NF; f += 64) S::template hrr_bra_col<1, double>(s_buf, f, bq.AB, s_abf);
            __syncthreads();
            for (int r = lane; r < NAB; r += 64) {
                double row[NCD];
                S::template hrr_ket_row<double>(s_abf + r * NF, kq.AB, row);
#pragma unroll
                for (int cd = 0; cd < NCD; ++cd) s_buf[r * NCD + cd] = row[cd];
            }
            __syncthreads();
            if (a.Q) {
                double mx = 0.0;
                for (int ab = lane; ab < NAB; ab += 64) mx = fmax(mx, s_buf[ab * NCD + ab]);
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
                if (lane == 0) a.Q[iq.bra] = sqrt(mx);
            } else {
                const bool sab = iq.flags & 1, scd = iq.flags & 2, sbk = iq.flags & 4;
                double *out = a.out + iq.out_off;
                for (int e = lane; e < NAB * NCD; e += 64) {
                    const int i = e / (NB * NCD), j = (e / NCD) % NB, k = (e % NCD) / ND, l = e % ND;
                    int x1, x2, x3, x4;
                    if (!sbk) {
                        x1 = sab ? j : i;
                        x2 = sab ? i : j;
                        x3 = scd ? l : k;
                        x4 = scd ? k : l;
                    } else {
                        x1 = sab ? l : k;
                        x2 = sab ? k : l;
                        x3 = scd ? j : i;
                        x4 = scd ? i : j;
                    }
                    out[((size_t)(x1 * iq.n2 + x2) * iq.n3 + x3) * iq.n4 + x4] = s_buf[e];
                }
            }
            __syncthreads();
        }
    }
}

// Occupancy bound of a persistent kernel: resident blocks per CU x CUs
// (-1 if the device cannot be queried).  The launch grid is this bound cut
// by persistent_blocks() to the staging slots and the work items.
template <typename K>
int occupancy_grid(K kernel, size_t lds)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu * ncu;
}

template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_jk_split(JKLaunch a)
{
    jk_split_body<LA, LB, LC, LD, T>(a);
}

// The FP32 split kernels need a little over 256 VGPRs; asking for two
// resident waves per SIMD trades a few spills for twice the occupancy.
template <int LA, int LB, int LC, int LD, typename T, int W>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W))) void k_jk_split_occ(JKLaunch a)
{
    jk_split_body<LA, LB, LC, LD, T>(a);
}

template <int LA, int LB, int LC, int LD, typename T>
int launch_split(const JKLaunch &a, hipStream_t s)
{
    if (a.nitems <= 0) return 0;
    constexpr bool OCC = sizeof(T) == sizeof(float);
    static int grid_cache = 0;  // occupancy bound, computed once
    if (grid_cache == 0) {
        if constexpr (OCC)
            grid_cache = occupancy_grid(k_jk_split_occ<LA, LB, LC, LD, T, 2>, 0);
        else
            grid_cache = occupancy_grid(k_jk_split<LA, LB, LC, LD, T>, 0);
        if (grid_cache <= 0) return kLaunchHip;
    }
    // every block stages one item's [e0|f0] in its own slot of NACC x 64 doubles
    const int64_t grid = persistent_blocks(grid_cache, a.nslot, a.nitems, true);
    if (grid < 1 || !staging_fits(grid, (int64_t)EriSplit<LA, LB, LC, LD>::NACC * 64, a.stage_bytes))
        return kLaunchStaging;
    if constexpr (OCC)
        hipLaunchKernelGGL((k_jk_split_occ<LA, LB, LC, LD, T, 2>), dim3((unsigned)grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_jk_split<LA, LB, LC, LD, T>), dim3((unsigned)grid), dim3(64), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : kLaunchHip;
}

template <int LA, int LB, int LC, int LD, typename T>
int launch_plain(const JKLaunch &a, hipStream_t s)
{
    if (a.nitems <= 0) return 0;
    constexpr int W = jk_waves<LA, LB, LC, LD>();
    static int grid_cache = 0;  // occupancy bound, computed once
    if (grid_cache == 0) {
        if constexpr (W > 0)
            grid_cache = occupancy_grid(k_jk_occ<LA, LB, LC, LD, T, W>, 0);
        else
            grid_cache = occupancy_grid(k_jk<LA, LB, LC, LD, T>, 0);
        if (grid_cache <= 0) return kLaunchHip;
    }
    const int64_t grid = a.lane_persistent ? persistent_blocks(grid_cache, 0, a.nitems, false) : a.nitems;
    if constexpr (W > 0)
        hipLaunchKernelGGL((k_jk_occ<LA, LB, LC, LD, T, W>), dim3((unsigned)grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_jk<LA, LB, LC, LD, T>), dim3((unsigned)grid), dim3(64), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : kLaunchHip;
}

template <int LA, int LB, int LC, int LD, typename T>
int launch_eri_split(const EriLaunch &a, hipStream_t s)
{
    if (a.n <= 0) return 0;
    static int grid_cache = 0;  // occupancy bound, computed once
    if (grid_cache == 0) {
        grid_cache = occupancy_grid(k_eri_split<LA, LB, LC, LD, T>, 0);
        if (grid_cache <= 0) return kLaunchHip;
    }
    const int64_t groups = a.deconstruct ? a.n : (a.n + 63) / 64;
    const int64_t grid = persistent_blocks(grid_cache, a.nslot, groups, true);
    if (grid < 1 || !staging_fits(grid, (int64_t)EriSplit<LA, LB, LC, LD>::NACC * 64, a.stage_bytes))
        return kLaunchStaging;
    hipLaunchKernelGGL((k_eri_split<LA, LB, LC, LD, T>), dim3((unsigned)grid), dim3(64), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : kLaunchHip;
}

// Classes with an f shell have no FP32 form: their "FP32" launchers run the
// FP64 kernels (the host never routes their quartets to FP32 lists).
template <int LA, int LB, int LC, int LD>
using fp32_of = std::conditional_t<(LA == 3 || LB == 3 || LC == 3 || LD == 3), double, float>;

// split classes: J/K launchers and eri_class / Schwarz launchers in separate
// translation units (they compile in parallel)
#define MJK_DEFINE_CLASS_SPLIT_JK(LA, LB, LC, LD, NAME)                                             \
    int launch_jk_##NAME(const JKLaunch &a, hipStream_t s)                                         \
    {                                                                                               \
        return launch_split<LA, LB, LC, LD, double>(a, s);                                          \
    }                                                                                               \
    int launch_jk32_##NAME(const JKLaunch &a, hipStream_t s)                                       \
    {                                                                                               \
        return launch_split<LA, LB, LC, LD, fp32_of<LA, LB, LC, LD>>(a, s);                         \
    }

#define MJK_DEFINE_CLASS_SPLIT_ERI(LA, LB, LC, LD, NAME)                                            \
    int launch_eri_##NAME(const EriLaunch &a, hipStream_t s)                                       \
    {                                                                                               \
        return launch_eri_split<LA, LB, LC, LD, double>(a, s);                                      \
    }                                                                                               \
    int launch_eri32_##NAME(const EriLaunch &a, hipStream_t s)                                     \
    {                                                                                               \
        return launch_eri_split<LA, LB, LC, LD, fp32_of<LA, LB, LC, LD>>(a, s);                     \
    }

#define MJK_DEFINE_CLASS(LA, LB, LC, LD, NAME)                                                      \
    int launch_jk_##NAME(const JKLaunch &a, hipStream_t s)                                         \
    {                                                                                               \
        return launch_plain<LA, LB, LC, LD, double>(a, s);                                          \
    }                                                                                               \
    int launch_jk32_##NAME(const JKLaunch &a, hipStream_t s)                                       \
    {                                                                                               \
        return launch_plain<LA, LB, LC, LD, float>(a, s);                                           \
    }                                                                                               \
    int launch_eri_##NAME(const EriLaunch &a, hipStream_t s)                                       \
    {                                                                                               \
        if (a.n <= 0) return 0;                                                                     \
        hipLaunchKernelGGL((k_eri<LA, LB, LC, LD, double>), dim3((a.n + 63) / 64), dim3(64), 0, s, a); \
        return hipGetLastError() == hipSuccess ? 0 : -1;                                            \
    }                                                                                               \
    int launch_eri32_##NAME(const EriLaunch &a, hipStream_t s)                                     \
    {                                                                                               \
        if (a.n <= 0) return 0;                                                                     \
        hipLaunchKernelGGL((k_eri<LA, LB, LC, LD, float>), dim3((a.n + 63) / 64), dim3(64), 0, s, a); \
        return hipGetLastError() == hipSuccess ? 0 : -1;                                            \
    }

#define MJK_DEFINE_SCHWARZ(LA, LB, NAME)                                                            \
    int launch_schwarz_##NAME(const SchwarzLaunch &a, hipStream_t s)                               \
    {                                                                                               \
        if (a.n <= 0) return 0;                                                                     \
        hipLaunchKernelGGL((k_schwarz<LA, LB>), dim3((a.n + 63) / 64), dim3(64), 0, s, a);          \
        return hipGetLastError() == hipSuccess ? 0 : -1;                                            \
    }

}  // namespace mjk
