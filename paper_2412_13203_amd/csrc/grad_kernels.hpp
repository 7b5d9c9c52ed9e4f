// grad_kernels.hpp -- nuclear gradient of E2 = 1/2 Tr(DJ) - 1/4 Tr(DK) at
// fixed density.
//
// Over unique shell quartets (weight w = 1/(s_AB s_CD s_ABCD), the same as
// the J/K digestion),
//   E2 = sum_quartets w sum_{abcd} (ab|cd) W_abcd,
//   W_abcd = 4 D_ab D_cd - D_ac D_bd - D_ad D_bc,
// so dE2/dR_X = sum_quartets w sum_{abcd} W_abcd d(ab|cd)/dX for the centres
// X = A, B, C; the fourth centre's derivative is minus their sum
// (translational invariance).  A Cartesian Gaussian moves with its centre:
//   d/dA_i phi_a = 2 alpha phi_{a+1_i} - a_i phi_{a-1_i},
// so d(ab|cd)/dA_i needs the class with la + 1 contracted with the primitive
// weight 2 alpha, and the class with la - 1 unweighted.  Each shifted class
// is an ordinary generated class: the weight scales the [00|00] prefactor,
// so contraction (Eq. 2) and the horizontal recurrence are unchanged.
//
// Work items are those of the J/K path (one bra pair x `chunk` kets, 64 at a
// time, one quartet per lane).  A shifted class whose accumulators fit a lane runs per
// lane; a larger one runs as passes into the staging slot, then the wave
// takes the quartets one at a time (bra HRR per ket column, ket HRR per (ab)
// row, contraction with W in LDS).  Gradient contributions go to a per-block
// copy of the gradient in LDS, flushed with one atomic per element at the end
// of the persistent block.  A launch covers the segments of one molecule.
#pragma once
#include "kernels.hpp"

namespace mjk {

// Cartesian component k of shell l (lexicographic: x descending, then y):
// its exponent along axis i.
__host__ __device__ constexpr int cart_pow(int l, int k, int i)
{
    int x = l;
    while (k > l - x) {  // components with this x: l - x + 1
        k -= l - x + 1;
        --x;
    }
    const int y = l - x - k, z = k;
    return i == 0 ? x : (i == 1 ? y : z);
}

// index of (x, y, z) inside shell l = x + y + z
__host__ __device__ constexpr int cart_at(int l, int x, int z) { return (l - x) * (l - x + 1) / 2 + z; }

// Component of shell l0 (the unshifted one) that component k of the shifted
// shell comes from, moving one step along axis i: -1 if none.  Up: the
// shifted shell is l0 + 1 and k = k0 + 1_i.  Down: l0 - 1 and k = k0 - 1_i.
__host__ __device__ constexpr int unshift(int l0, bool up, int k, int i)
{
    const int ls = up ? l0 + 1 : l0 - 1;
    int x = cart_pow(ls, k, 0), z = cart_pow(ls, k, 2);
    const int p = cart_pow(ls, k, i);
    if (up && p == 0) return -1;
    const int d = up ? -1 : 1;
    if (i == 0) x += d;
    if (i == 2) z += d;
    return cart_at(l0, x, z);
}

// the factor in front of the shifted integral: 1 for the raised class
// (its 2 alpha is inside the contraction), -k0_i for the lowered one
__host__ __device__ constexpr double shift_coef(int l0, bool up, int k, int i)
{
    if (up) return 1.0;
    return -(double)(cart_pow(l0 - 1, k, i) + 1);
}

template <int LA, int LB, int LC, int LD, int S>
struct GradSub {
    static constexpr int CEN = S / 2;  // 0: A, 1: B, 2: C
    static constexpr bool UP = (S % 2) == 0;
    static constexpr int D = UP ? 1 : -1;
    static constexpr int SLA = LA + (CEN == 0 ? D : 0);
    static constexpr int SLB = LB + (CEN == 1 ? D : 0);
    static constexpr int SLC = LC + (CEN == 2 ? D : 0);
    static constexpr int SLD = LD;
    static constexpr bool VALID = SLA >= 0 && SLB >= 0 && SLC >= 0;
    static constexpr int WK = UP ? (CEN == 0 ? WK_A : (CEN == 1 ? WK_B : WK_C)) : WK_ONE;
};

// A shifted class runs one quartet per lane when its accumulators and its
// Cartesian block together fit this many doubles; larger ones run through
// the staging slot and the cooperative HRR.  Measured on the 60-atom
// gradient: 40 -> 96 -> 128 took the backward from 8.81 to 8.29 to 7.90 s
// (per-lane runs win even where they spill a little; nothing changes above 128).
constexpr int kGradLaneMax = 128;

template <int LA, int LB, int LC, int LD, int S>
constexpr bool grad_sub_split()
{
    using G = GradSub<LA, LB, LC, LD, S>;
    if constexpr (G::VALID) {
        using C = EriClass<G::SLA, G::SLB, G::SLC, G::SLD>;
        return C::SPLIT || C::NACC + C::NOUT > kGradLaneMax;
    } else {
        return false;
    }
}

template <int LA, int LB, int LC, int LD, int S>
constexpr size_t grad_sub_nacc()
{
    using G = GradSub<LA, LB, LC, LD, S>;
    if constexpr (grad_sub_split<LA, LB, LC, LD, S>())
        return (size_t)EriSplit<G::SLA, G::SLB, G::SLC, G::SLD>::NACC;
    else
        return 0;
}

// staging doubles per lane needed by the split shifted classes of a class
template <int LA, int LB, int LC, int LD>
constexpr size_t grad_stage_nacc()
{
    size_t m = 0;
    const size_t v[6] = {grad_sub_nacc<LA, LB, LC, LD, 0>(), grad_sub_nacc<LA, LB, LC, LD, 1>(),
                         grad_sub_nacc<LA, LB, LC, LD, 2>(), grad_sub_nacc<LA, LB, LC, LD, 3>(),
                         grad_sub_nacc<LA, LB, LC, LD, 4>(), grad_sub_nacc<LA, LB, LC, LD, 5>()};
    for (int i = 0; i < 6; ++i) m = v[i] > m ? v[i] : m;
    return m;
}

// largest (ab) row count x ket column count of the split shifted classes
template <int LA, int LB, int LC, int LD, int S>
constexpr int grad_sub_abf()
{
    using G = GradSub<LA, LB, LC, LD, S>;
    if constexpr (grad_sub_split<LA, LB, LC, LD, S>())
        return ncart(G::SLA) * ncart(G::SLB) * EriSplit<G::SLA, G::SLB, G::SLC, G::SLD>::NF;
    else
        return 1;
}

template <int LA, int LB, int LC, int LD>
constexpr int grad_abf_max()
{
    const int v[6] = {grad_sub_abf<LA, LB, LC, LD, 0>(), grad_sub_abf<LA, LB, LC, LD, 1>(),
                      grad_sub_abf<LA, LB, LC, LD, 2>(), grad_sub_abf<LA, LB, LC, LD, 3>(),
                      grad_sub_abf<LA, LB, LC, LD, 4>(), grad_sub_abf<LA, LB, LC, LD, 5>()};
    int m = 1;
    for (int i = 0; i < 6; ++i) m = v[i] > m ? v[i] : m;
    return m;
}

template <int LA, int LB, int LC, int LD>
constexpr bool grad_any_split()
{
    return grad_sub_split<LA, LB, LC, LD, 0>() || grad_sub_split<LA, LB, LC, LD, 1>() ||
           grad_sub_split<LA, LB, LC, LD, 2>() || grad_sub_split<LA, LB, LC, LD, 3>() ||
           grad_sub_split<LA, LB, LC, LD, 4>() || grad_sub_split<LA, LB, LC, LD, 5>();
}

// Density weights of one quartet, W_abcd = 4 D_ab D_cd - D_ac D_bd - D_ad D_bc,
// read from D (row-major N x N).
struct QuartetAO {
    int a, b, c, d;  // first AO of each shell
};

__device__ __forceinline__ double wdens(gptr<double> __restrict__ D, int N, const QuartetAO &o, int ia, int jb,
                                        int kc, int ld)
{
    const double dab = D[(size_t)(o.a + ia) * N + o.b + jb], dcd = D[(size_t)(o.c + kc) * N + o.d + ld];
    const double dac = D[(size_t)(o.a + ia) * N + o.c + kc], dbd = D[(size_t)(o.b + jb) * N + o.d + ld];
    const double dad = D[(size_t)(o.a + ia) * N + o.d + ld], dbc = D[(size_t)(o.b + jb) * N + o.c + kc];
    return 4.0 * dab * dcd - dac * dbd - dad * dbc;
}

// W of one quartet in registers when it is this small (else read from D
// per use, which the unrolled code keeps in cache)
constexpr int kGradWRegMax = 36;

// One shifted class, one quartet per lane: contraction with its primitive
// weight, HRR, and the contraction of the shifted block with W into the
// three Cartesian components of the shifted centre's derivative.
template <int LA, int LB, int LC, int LD, int S>
__device__ __forceinline__ void grad_sub_lane(const ShellPairD &bra, const ShellPairD &ket,
                                              const PrimPairD *__restrict__ prims, bool active,
                                              gptr<double> __restrict__ D, int N, const QuartetAO &o,
                                              const double *Wr, double g[3])
{
    using G = GradSub<LA, LB, LC, LD, S>;
    using C = EriClass<G::SLA, G::SLB, G::SLC, G::SLD>;
    constexpr int L = G::SLA + G::SLB + G::SLC + G::SLD;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int SA = ncart(G::SLA), SB = ncart(G::SLB), SC = ncart(G::SLC), SD = ncart(G::SLD);
    double acc[C::NACC];
#pragma unroll
    for (int i = 0; i < C::NACC; ++i) acc[i] = 0.0;
    prim_loop<L, G::WK>(bra, ket, prims, active,
                        [&](const double *F, const VrrGeom<double> &gm) { C::template vrr<double>(F, gm, acc); });
    double eri[C::NOUT];
    C::template hrr<double>(acc, bra.AB, ket.AB, eri);
#pragma unroll
    for (int ia = 0; ia < SA; ++ia)
#pragma unroll
        for (int jb = 0; jb < SB; ++jb)
#pragma unroll
            for (int kc = 0; kc < SC; ++kc)
#pragma unroll
                for (int ld = 0; ld < SD; ++ld) {
                    const double v = eri[((ia * SB + jb) * SC + kc) * SD + ld];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        int a = ia, b = jb, c = kc;
                        double cf;
                        if constexpr (G::CEN == 0) {
                            a = unshift(LA, G::UP, ia, i);
                            cf = shift_coef(LA, G::UP, ia, i);
                        } else if constexpr (G::CEN == 1) {
                            b = unshift(LB, G::UP, jb, i);
                            cf = shift_coef(LB, G::UP, jb, i);
                        } else {
                            c = unshift(LC, G::UP, kc, i);
                            cf = shift_coef(LC, G::UP, kc, i);
                        }
                        if (a >= 0 && b >= 0 && c >= 0) {
                            double wv;
                            if constexpr (NA * NB * NC * ND <= kGradWRegMax)
                                wv = Wr[((a * NB + b) * NC + c) * ND + ld];
                            else
                                wv = wdens(D, N, o, a, b, c, ld);
                            g[i] += cf * v * wv;
                        }
                    }
                }
}

template <int LA, int LB, int LC, int LD, int S>
__device__ __forceinline__ void grad_sub_lane_if(const ShellPairD &bra, const ShellPairD &ket,
                                                 const PrimPairD *__restrict__ prims, bool active,
                                                 gptr<double> __restrict__ D, int N, const QuartetAO &o,
                                                 const double *Wr, double gA[3], double gB[3], double gC[3])
{
    using G = GradSub<LA, LB, LC, LD, S>;
    if constexpr (G::VALID && !grad_sub_split<LA, LB, LC, LD, S>()) {
        double *g = G::CEN == 0 ? gA : (G::CEN == 1 ? gB : gC);
        grad_sub_lane<LA, LB, LC, LD, S>(bra, ket, prims, active, D, N, o, Wr, g);
    }
}

template <int LA, int LB, int LC, int LD, int S>
constexpr bool grad_sub_lane_used()
{
    return GradSub<LA, LB, LC, LD, S>::VALID && !grad_sub_split<LA, LB, LC, LD, S>();
}

// One split shifted class for the item's quartets: passes into the staging
// slot, then per quartet the cooperative HRR and the contraction with W.
// The derivative of quartet q is added to lane q's g (times its weight).
template <int LA, int LB, int LC, int LD, int S>
__device__ __forceinline__ void grad_sub_split_run(const ShellPairD &bra, const ShellPairD &ket,
                                                   const PrimPairD *__restrict__ prims, bool active,
                                                   gptr<double> __restrict__ D, int N, int nact, int lane,
                                                   double *__restrict__ stage, double *__restrict__ s_abf,
                                                   double *__restrict__ s_W, const double *s_w, const double (*s_CD)[3],
                                                   const int (*s_ao)[2], double gA[3], double gB[3], double gC[3])
{
    using G = GradSub<LA, LB, LC, LD, S>;
    if constexpr (G::VALID && grad_sub_split<LA, LB, LC, LD, S>()) {
        using SP = EriSplit<G::SLA, G::SLB, G::SLC, G::SLD>;
        constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
        constexpr int NCD = NC * ND, NW = NA * NB * NCD;
        constexpr int SA = ncart(G::SLA), SB = ncart(G::SLB), SC = ncart(G::SLC);
        constexpr int SAB = SA * SB, SCD = SC * ND, NF = SP::NF;
        split_passes<G::SLA, G::SLB, G::SLC, G::SLD, 0, double, G::WK>(bra, ket, prims, active, stage, lane);
        __syncthreads();
        double *g = G::CEN == 0 ? gA : (G::CEN == 1 ? gB : gC);
        for (int q = 0; q < nact; ++q) {
            const QuartetAO o{bra.ao_a, bra.ao_b, s_ao[q][0], s_ao[q][1]};
            for (int t = lane; t < NW; t += 64) {
                const int ab = t / NCD, cd = t % NCD;
                s_W[t] = wdens(D, N, o, ab / NB, ab % NB, cd / ND, cd % ND);
            }
            // bra HRR straight from the staging slot ([target][lane] layout)
            for (int f = lane; f < NF; f += 64)
                SP::template hrr_bra_col<64, double>(stage + q, f, bra.AB, s_abf);
            __syncthreads();
            const double CD[3] = {s_CD[q][0], s_CD[q][1], s_CD[q][2]};
            double t0 = 0.0, t1 = 0.0, t2 = 0.0;
            for (int r = lane; r < SAB; r += 64) {
                double row[SCD];
                SP::template hrr_ket_row<double>(s_abf + r * NF, CD, row);
                if constexpr (G::CEN == 2) {
                    // ket shift: row r is the unshifted (ab)
#pragma unroll
                    for (int kc = 0; kc < SC; ++kc)
#pragma unroll
                        for (int ld = 0; ld < ND; ++ld) {
                            const double v = row[kc * ND + ld];
                            const int c0 = unshift(LC, G::UP, kc, 0), c1 = unshift(LC, G::UP, kc, 1),
                                      c2 = unshift(LC, G::UP, kc, 2);
                            if (c0 >= 0) t0 += shift_coef(LC, G::UP, kc, 0) * v * s_W[r * NCD + c0 * ND + ld];
                            if (c1 >= 0) t1 += shift_coef(LC, G::UP, kc, 1) * v * s_W[r * NCD + c1 * ND + ld];
                            if (c2 >= 0) t2 += shift_coef(LC, G::UP, kc, 2) * v * s_W[r * NCD + c2 * ND + ld];
                        }
                } else {
                    // bra shift: the unshifted (ab) row depends on the direction
                    const int ia = r / SB, jb = r % SB;
                    double tt[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        int a = ia, b = jb;
                        double cf;
                        if constexpr (G::CEN == 0) {
                            a = unshift(LA, G::UP, ia, i);
                            cf = shift_coef(LA, G::UP, ia, i);
                        } else {
                            b = unshift(LB, G::UP, jb, i);
                            cf = shift_coef(LB, G::UP, jb, i);
                        }
                        double s = 0.0;
                        if (a >= 0 && b >= 0) {
                            const double *wr = s_W + (a * NB + b) * NCD;
#pragma unroll
                            for (int cd = 0; cd < NCD; ++cd) s += row[cd] * wr[cd];
                        }
                        tt[i] = cf * s;
                    }
                    t0 += tt[0];
                    t1 += tt[1];
                    t2 += tt[2];
                }
            }
            t0 = wave_sum(t0);
            t1 = wave_sum(t1);
            t2 = wave_sum(t2);
            if (lane == q) {
                const double w = s_w[q];
                g[0] += w * t0;
                g[1] += w * t1;
                g[2] += w * t2;
            }
            __syncthreads();
        }
    }
}

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(64) void k_grad(JKLaunch a)
{
    constexpr bool ANY_SPLIT = grad_any_split<LA, LB, LC, LD>();
    constexpr int NW = ncart(LA) * ncart(LB) * ncart(LC) * ncart(LD);
    constexpr int NABF = grad_abf_max<LA, LB, LC, LD>();
    __shared__ double s_abf[ANY_SPLIT ? NABF : 1];
    __shared__ double s_W[ANY_SPLIT ? NW : 1];
    __shared__ double s_CD[64][3];
    __shared__ double s_w[64];
    __shared__ int s_ao[64][2];
    extern __shared__ double s_g[];  // the molecule's gradient (natom x 3), this block's share
    const int lane = threadIdx.x;
    const int n3 = 3 * a.natom_max;
    double *stage = a.stage + (size_t)blockIdx.x * grad_stage_nacc<LA, LB, LC, LD>() * 64;
    for (int t = lane; t < n3; t += 64) s_g[t] = 0.0;
    __syncthreads();

    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const JKSeg sg = ldg(a.segs + find_seg(a, item));
        int b, kbeg, kend;
        locate(sg, item - sg.item_begin, b, kbeg, kend);
        const int bra_pos = sg.bra_begin + b;
        const ShellPairD bra = ldg(sg.pairs + bra_pos);
        const int N = sg.nbf;
        const gptr<double> __restrict__ D = gview(a.D + sg.mat_off);
        const int atA = ldg(sg.shell_atom + bra.A), atB = ldg(sg.shell_atom + bra.B);
        double bA[3] = {0.0, 0.0, 0.0}, bB[3] = {0.0, 0.0, 0.0};  // bra centres, summed over the item
        int run = find_run(sg, b, kbeg);
        const int run_end = ldg(sg.run_begin + b + 1);

        for (int k0 = kbeg; k0 < kend; k0 += 64) {
            const int nact = min(kend - k0, 64);
            const bool active = lane < nact;
            const RoundKets rk = round_kets(sg, run, run_end, k0, lane);
            const int pos0 = __builtin_amdgcn_readfirstlane(__shfl(rk.pos, 0, 64));
            const int ket_pos = sg.ket_begin + (active ? rk.pos : pos0);
            const ShellPairD ket = ldg(sg.pairs + ket_pos);
            double s = 1.0;
            if (bra.same) s *= 2.0;
            if (ket.same) s *= 2.0;
            if (sg.same_bin && ket_pos == bra_pos) s *= 2.0;
            const double w = active ? 1.0 / s : 0.0;
            s_w[lane] = w;
            s_CD[lane][0] = ket.AB[0];
            s_CD[lane][1] = ket.AB[1];
            s_CD[lane][2] = ket.AB[2];
            s_ao[lane][0] = ket.ao_a;
            s_ao[lane][1] = ket.ao_b;
            const QuartetAO o{bra.ao_a, bra.ao_b, ket.ao_a, ket.ao_b};

            double gA[3] = {0.0, 0.0, 0.0}, gB[3] = {0.0, 0.0, 0.0}, gC[3] = {0.0, 0.0, 0.0};
            {
                // per-lane shifted classes, weighted by this lane's w at the end
                double lA[3] = {0.0, 0.0, 0.0}, lB[3] = {0.0, 0.0, 0.0}, lC[3] = {0.0, 0.0, 0.0};
                constexpr bool ANY_LANE =
                    grad_sub_lane_used<LA, LB, LC, LD, 0>() || grad_sub_lane_used<LA, LB, LC, LD, 1>() ||
                    grad_sub_lane_used<LA, LB, LC, LD, 2>() || grad_sub_lane_used<LA, LB, LC, LD, 3>() ||
                    grad_sub_lane_used<LA, LB, LC, LD, 4>() || grad_sub_lane_used<LA, LB, LC, LD, 5>();
                constexpr int NWR = (ANY_LANE && NW <= kGradWRegMax) ? NW : 1;
                double Wr[NWR];
                if constexpr (ANY_LANE && NW <= kGradWRegMax) {
                    constexpr int NB_ = ncart(LB), NC_ = ncart(LC), ND_ = ncart(LD);
#pragma unroll
                    for (int t = 0; t < NW; ++t)
                        Wr[t] = wdens(D, N, o, t / (NB_ * NC_ * ND_), (t / (NC_ * ND_)) % NB_, (t / ND_) % NC_,
                                      t % ND_);
                }
                grad_sub_lane_if<LA, LB, LC, LD, 0>(bra, ket, sg.prims, active, D, N, o, Wr, lA, lB, lC);
                grad_sub_lane_if<LA, LB, LC, LD, 1>(bra, ket, sg.prims, active, D, N, o, Wr, lA, lB, lC);
                grad_sub_lane_if<LA, LB, LC, LD, 2>(bra, ket, sg.prims, active, D, N, o, Wr, lA, lB, lC);
                grad_sub_lane_if<LA, LB, LC, LD, 3>(bra, ket, sg.prims, active, D, N, o, Wr, lA, lB, lC);
                grad_sub_lane_if<LA, LB, LC, LD, 4>(bra, ket, sg.prims, active, D, N, o, Wr, lA, lB, lC);
                grad_sub_lane_if<LA, LB, LC, LD, 5>(bra, ket, sg.prims, active, D, N, o, Wr, lA, lB, lC);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    gA[i] = w * lA[i];
                    gB[i] = w * lB[i];
                    gC[i] = w * lC[i];
                }
            }
            if constexpr (ANY_SPLIT) {
                __syncthreads();  // s_w, s_CD, s_ao of this round
                grad_sub_split_run<LA, LB, LC, LD, 0>(bra, ket, sg.prims, active, D, N, nact, lane, stage, s_abf,
                                                      s_W, s_w, s_CD, s_ao, gA, gB, gC);
                grad_sub_split_run<LA, LB, LC, LD, 1>(bra, ket, sg.prims, active, D, N, nact, lane, stage, s_abf,
                                                      s_W, s_w, s_CD, s_ao, gA, gB, gC);
                grad_sub_split_run<LA, LB, LC, LD, 2>(bra, ket, sg.prims, active, D, N, nact, lane, stage, s_abf,
                                                      s_W, s_w, s_CD, s_ao, gA, gB, gC);
                grad_sub_split_run<LA, LB, LC, LD, 3>(bra, ket, sg.prims, active, D, N, nact, lane, stage, s_abf,
                                                      s_W, s_w, s_CD, s_ao, gA, gB, gC);
                grad_sub_split_run<LA, LB, LC, LD, 4>(bra, ket, sg.prims, active, D, N, nact, lane, stage, s_abf,
                                                      s_W, s_w, s_CD, s_ao, gA, gB, gC);
                grad_sub_split_run<LA, LB, LC, LD, 5>(bra, ket, sg.prims, active, D, N, nact, lane, stage, s_abf,
                                                      s_W, s_w, s_CD, s_ao, gA, gB, gC);
            }
            if (active) {
                const int atC = ldg(sg.shell_atom + ket.A), atD = ldg(sg.shell_atom + ket.B);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    atomicAdd(&s_g[3 * atC + i], gC[i]);
                    atomicAdd(&s_g[3 * atD + i], -(gA[i] + gB[i] + gC[i]));
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                bA[i] += gA[i];
                bB[i] += gB[i];
            }
            __syncthreads();  // LDS of this round is reused by the next
        }
        // bra centres are shared by the item: reduce over the wave first
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double sa = wave_sum(bA[i]), sb = wave_sum(bB[i]);
            if (lane == 0) {
                atomicAdd(&s_g[3 * atA + i], sa);
                atomicAdd(&s_g[3 * atB + i], sb);
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (int t = lane; t < n3; t += 64) {
        const double v = s_g[t];
        if (v != 0.0) atomicAdd(a.grad + t, v);
    }
}

template <int LA, int LB, int LC, int LD>
int launch_grad(const JKLaunch &a, hipStream_t s)
{
    if (a.nitems <= 0) return 0;
    const size_t lds = sizeof(double) * 3 * (size_t)a.natom_max;
    static size_t cached_lds = (size_t)-1;
    static int grid_cache = 0;
    if (cached_lds != lds) {
        grid_cache = occupancy_grid(k_grad<LA, LB, LC, LD>, lds);
        if (grid_cache <= 0) return kLaunchHip;
        cached_lds = lds;
    }
    // a block with split shifted classes stages them in its own slot of
    // grad_stage_nacc x 64 doubles (blocks stride over the items)
    constexpr int64_t slot = (int64_t)grad_stage_nacc<LA, LB, LC, LD>() * 64;
    const int64_t grid = persistent_blocks(grid_cache, a.nslot, a.nitems, slot > 0);
    if (grid < 1 || !staging_fits(grid, slot, a.stage_bytes)) return kLaunchStaging;
    hipLaunchKernelGGL((k_grad<LA, LB, LC, LD>), dim3((unsigned)grid), dim3(64), lds, s, a);
    return hipGetLastError() == hipSuccess ? 0 : kLaunchHip;
}

#define MJK_DEFINE_GRAD(LA, LB, LC, LD, NAME)                                                       \
    int launch_grad_##NAME(const JKLaunch &a, hipStream_t s) { return launch_grad<LA, LB, LC, LD>(a, s); } \
    size_t grad_stage_nacc_##NAME() { return grad_stage_nacc<LA, LB, LC, LD>(); }

}  // namespace mjk
