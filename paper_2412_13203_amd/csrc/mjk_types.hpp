// mjk_types.hpp -- data laid out in device memory and the launch records
// passed from the host planner to the class kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mjk {

// One primitive pair (alpha on the first centre A, beta on the second B),
// 80 bytes.  K folds the coefficients, the Gaussian product factor and the
// pair part of the [00|00] prefactor:
//   K = sqrt(2) pi^{5/4} c_a c_b exp(-alpha beta / p |AB|^2) / p,
// so that K_bra K_ket / sqrt(p + q) = 2 pi^{5/2} / (p q sqrt(p+q)) * ...
struct alignas(16) PrimPairD {
    double p;        // alpha + beta
    double oo2p;     // 1 / (2p)
    double P[3];     // (alpha A + beta B) / p
    double PA[3];    // P - A
    double K;
    double alpha;    // exponent of the first centre (derivative integrals)
};
static_assert(sizeof(PrimPairD) == 80, "PrimPairD layout");

// One shell pair, oriented so that l(A) >= l(B); 64 bytes.
struct alignas(16) ShellPairD {
    int32_t A, B;          // shell indices (first, second centre)
    int32_t prim_off;      // first primitive pair in the primitive-pair table
    int32_t nprim;         // K_A * K_B (A-major)
    int32_t ao_a, ao_b;    // first AO index of A and of B
    int32_t same;          // 1 if A == B (identical shells)
    int32_t cls;           // pair class index la(la+1)/2 + lb
    double AB[3];          // A - B
    double Q;              // Schwarz factor
};
static_assert(sizeof(ShellPairD) == 64, "ShellPairD layout");

// Explicit quartet for the eri_class path.
struct alignas(16) EriItem {
    int32_t bra, ket;      // pair indices in the natural pair table
    int32_t flags;         // bit0: swap a<->b, bit1: swap c<->d, bit2: swap bra<->ket
    int32_t pad;
    int64_t out_off;       // first output element of this quartet
    int32_t n1, n2, n3, n4;// caller's component counts (A, B, C, D)
};

// One kept run of a bra's ket list.  Inside a bin the pairs are ordered by
// their first shell C, then by Schwarz factor (descending); a run is the
// pairs of one C.  A bra keeps a prefix of every run (screening and, when the
// bra and ket bins coincide, the ket <= bra triangle both cut prefixes), so
// its kets, numbered 0, 1, ... in run order, are described by the runs it
// keeps: run r holds kets [start_r, start_{r+1}) beginning at bin position pos_r.
struct KetRun {
    int32_t start;               // first ket number of the run (per bra, per precision)
    int32_t pos;                 // bin position of that ket
};

// One segment of a class launch: the quartets of one (bra bin, ket bin) pair
// of one molecule at one precision.  Work items of a launch are numbered
// across its segments (item_begin); an item is one bra pair x `chunk` kets.
struct alignas(16) JKSeg {
    const ShellPairD *pairs;     // the molecule's class-sorted pair table
    const PrimPairD *prims;
    const KetRun *runs;          // the molecule's kept-run table
    const int32_t *ket_count;    // per bra: kept kets
    const int32_t *run_begin;    // per bra: first kept run (nbra + 1, into runs)
    const int32_t *chunk_prefix; // per bra: exclusive prefix of chunks (nbra + 1)
    const int32_t *shell_atom;   // gradient: atom of each shell
    int64_t mat_off;             // first element of this molecule's D, J, K
    int32_t nbf, bra_begin, nbra, ket_begin;
    int32_t same_bin;            // bra and ket bins coincide: keep ket <= bra
    int32_t chunk;               // kets per item (multiple of 64)
    int32_t item_begin;          // first launch item of this segment
    int32_t mol;                 // molecule index
    int32_t grad_off;            // gradient: first element of this molecule's gradient
    int32_t natom;
};

struct JKLaunch {
    const JKSeg *segs;           // device array, item_begin ascending
    int32_t nseg;
    int32_t nitems;              // items over all segments
    const double *D;             // molecule m's matrices start at segs[].mat_off
    double *J;
    double *K;
    double *grad;                // gradient launches only
    double *stage;               // split classes: per-slot staging of [e0|f0]
    size_t stage_bytes;          // size of the staging region at `stage`
    int32_t nslot;               // split classes: staging slots (persistent blocks)
    int32_t natom_max;           // gradient: LDS copy of one molecule's gradient
    uint32_t *queue;             // persistent kernels: work counter, zero at launch
    unsigned long long *stamps;  // optional: per molecule [first start, last end]
    int32_t lane_persistent;     // per-lane classes: persistent waves pop items (else one block per item)
};

struct EriLaunch {
    const ShellPairD *pairs;   // natural pair table
    const PrimPairD *prims;
    const EriItem *items;
    int32_t n;
    double *out;
    // split classes: per-block staging slots of [e0|f0] (persistent blocks)
    double *stage;
    size_t stage_bytes;
    int32_t nslot;
    // Schwarz mode (split diagonal classes): items are (pair, pair) and
    // Q[bra] = sqrt(max_{a,b} (ab|ab)) is written instead of `out`
    double *Q;
    // split classes: one quartet per block, its primitive quartets spread
    // over the lanes (for few quartets with many primitives each)
    int32_t deconstruct;
};

struct SchwarzLaunch {
    const ShellPairD *pairs;   // natural pair table
    const PrimPairD *prims;
    const int32_t *idx;        // natural pair indices of one pair class
    int32_t n;
    double *Q;                 // natural order
};

using JKFn = int (*)(const JKLaunch &, hipStream_t);
using EriFn = int (*)(const EriLaunch &, hipStream_t);
using SchwarzFn = int (*)(const SchwarzLaunch &, hipStream_t);

struct ClassEntry {
    int la, lb, lc, ld;
    int nacc, nout;
    double vrr_flops;  // per primitive quartet (all passes of a split class)
    double hrr_flops;  // per contracted quartet
    int split;         // 1: multi-pass VRR + cooperative HRR/digestion
    int npass;
    JKFn jk;
    JKFn jk32;         // FP32 recurrence / contraction, FP64 digestion
    EriFn eri;
    EriFn eri32;        // FP32 recurrence / contraction, FP64 HRR
    SchwarzFn schwarz;  // only on diagonal classes (la lb | la lb)
    // nuclear gradient: shifted classes (d/dA, d/dB, d/dC raise or lower one
    // centre), their staging need and algorithmic work
    JKFn grad;
    size_t (*grad_stage_nacc)();
    double grad_vrr_flops;  // per primitive quartet, all shifted classes
    int grad_nup, grad_ndown;  // shifted classes with L+1 and with L-1
    double grad_q_flops;    // per contracted quartet: HRR + contraction with D
};

}  // namespace mjk
