/*
 * mjk.h -- C ABI of the MI355X (gfx950) library that evaluates two-electron
 * repulsion integrals (ERIs) over contracted Cartesian Gaussian shells and
 * contracts them at once with a density matrix into the Coulomb (J) and
 * exchange (K) matrices.
 *
 * Problem statement (arXiv 2412.13203, Sections 2.1-2.2):
 *   - a contracted basis function is a fixed linear combination of primitive
 *     Cartesian Gaussians sharing one angular momentum (Eq. 1);
 *   - a contracted ERI (ab|cd) is the sum over primitive quartets of the
 *     coefficient products times the primitive integrals (Eq. 2), evaluated
 *     by horizontal and vertical recurrences down to an analytic [00|00];
 *   - the SCF loop builds the two-electron part of the Fock matrix from the
 *     current density at every iteration (Section 2.1):
 *         J_mn = sum_ls (mn|ls) D_ls,   K_mn = sum_ls (ml|ns) D_ls.
 *
 * Conventions shared by every call:
 *   - Units are bohr.  Real Cartesian functions, chemists' notation.
 *   - Shells: l in 0..mjk_lmax() (3 in the default build), 1..6 primitives.  The
 *     nuclear gradient takes l <= mjk_grad_lmax().  Coefficients are final: they
 *     multiply the unnormalized primitive x^i y^j z^k exp(-alpha r^2); the
 *     library never normalizes.
 *   - AO order: shells in input order; inside a shell the Cartesian
 *     components are lexicographic (d: xx xy xz yy yz zz; f: xxx xxy xxz xyy
 *     xyz xzz yyy yyz yzz zzz).  Matrices are nbf x nbf row-major float64.
 *   - Device pointers (D, J, K, out, workspace) are caller-owned memory on
 *     the context's device, e.g. contiguous torch tensors.  Host pointers are
 *     read during the call only (basis arrays: during mjk_plan_create).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work calls are asynchronous on it unless stated otherwise.
 *   - Every function returns an int status: MJK_OK (0) or a negative error
 *     code; mjk_last_error() gives the message of the last failure on the
 *     calling thread, mjk_ctx_last_error(ctx) that of the last failed call
 *     made with a context (directly or through its plans and batches).  No
 *     exception crosses the ABI.  Arguments are checked on the host before
 *     any launch; a device fault surfaces at the next call that synchronizes.
 */
#ifndef MJK_H
#define MJK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MJK_OK 0
#define MJK_ERR_INVALID_ARG (-1)  /* null pointer, bad index, bad size, non-finite input  */
#define MJK_ERR_UNSUPPORTED (-2)  /* l > lmax of the build, nprim outside 1..6            */
#define MJK_ERR_NO_DEVICE (-3)    /* no HIP device, or not a gfx950 device                */
#define MJK_ERR_WORKSPACE (-4)    /* workspace pointer null, misaligned or too small      */
#define MJK_ERR_HIP (-5)          /* a HIP runtime call failed                            */
#define MJK_ERR_STATE (-6)        /* call out of order (e.g. build before bind), or a      *
                                   * staging region too small for a launch's blocks       */

/* Flags of mjk_jk_opts.flags */
#define MJK_FLAG_CHECK 0x1u       /* check D on the host side of the call: finite and symmetric */
#define MJK_FLAG_GRAD 0x2u        /* size the workspace for mjk_grad_e2 as well                 */
#define MJK_FLAG_NO_STAGING 0x4u  /* no staging slots or work counters in the workspace: the plan
                                   * builds J and K with mjk_build_jk_static only (not with
                                   * MJK_FLAG_GRAD, not in batches)                              */
#define MJK_FLAG_NO_KBINS 0x10u   /* ablation of the binning: shell pairs of one angular-momentum
                                   * class share one bin whatever their primitive-pair count    */
#define MJK_FLAG_PERSISTENT 0x8u  /* J/K builds: the per-lane classes run persistent waves that
                                   * take work items from the launch's counter (the split classes
                                   * always do); without it, one block per work item             */

typedef struct mjk_ctx mjk_ctx;
typedef struct mjk_plan mjk_plan;

/* Contracted basis on atoms (host memory, read by mjk_plan_create only).
 * Eq. 1: shell s is sum_k coefs[prim_off+k] * primitive(exps[prim_off+k]),
 * k < shell_nprim[s], centred on atom shell_atom[s]. */
typedef struct mjk_basis {
    int32_t natom;
    const double *xyz;            /* natom x 3, bohr                         */
    int32_t nshell;
    const int32_t *shell_atom;    /* nshell, 0..natom-1                      */
    const int32_t *shell_l;       /* nshell, 0..mjk_lmax()                   */
    const int32_t *shell_nprim;   /* nshell, 1..6                            */
    const int32_t *shell_prim_off;/* nshell, offset into exps / coefs        */
    int64_t nprim;                /* length of exps and coefs                */
    const double *exps;           /* > 0, finite                             */
    const double *coefs;          /* finite                                  */
} mjk_basis;

/* Options of a plan.
 * schwarz_tau: a unique shell quartet (AB|CD) is skipped iff
 *   Q_AB * Q_CD < schwarz_tau, with Q_AB = sqrt(max_{a in A, b in B} (ab|ab))
 *   (Cauchy-Schwarz bound; 0 keeps every quartet).
 * fp32_tau: mixed precision.  A kept quartet with Q_AB * Q_CD < fp32_tau
 *   runs its vertical recurrence and its contraction over primitives in FP32
 *   (the geometry and Boys function are evaluated in FP64 and rounded); the
 *   horizontal recurrence and the digestion into J and K run in FP64.
 *   0 = every quartet in FP64. */
typedef struct mjk_jk_opts {
    double schwarz_tau;
    double fp32_tau;
    uint32_t flags;
} mjk_jk_opts;

/* Plan statistics (filled after mjk_plan_bind). */
typedef struct mjk_plan_stats {
    int64_t nbf;
    int64_t nshell;
    int64_t npair;              /* shell pairs A >= B                              */
    int64_t nprim_pair;         /* primitive pairs over all shell pairs            */
    int64_t nquartet_total;     /* unique shell quartets before screening          */
    int64_t nquartet_kept;      /* unique shell quartets after screening           */
    int64_t nquartet_fp32;      /* kept quartets run in FP32 (fp32_tau)            */
    int64_t nprim_quartet_kept; /* primitive quartets of the kept quartets         */
    int64_t ncart_eri_kept;     /* Cartesian integrals of the kept quartets        */
    int64_t nlaunch;            /* kernel launches per mjk_build_jk                */
    double vrr_flops_kept;      /* algorithmic flops of the kept quartets          */
    size_t workspace_bytes;
    double grad_flops_kept;     /* algorithmic flops of mjk_grad_e2 (MJK_FLAG_GRAD) */
} mjk_plan_stats;

/* Library identification: lmax of the build (highest shell l supported by
 * the J/K build, eri_class and the Schwarz factors) and the highest shell l
 * the nuclear gradient supports (its shifted classes reach one more). */
int mjk_lmax(void);
int mjk_grad_lmax(void);

/* Quartet classes of the build: classes (la lb | lc ld) with la >= lb,
 * lc >= ld and pair class (la, lb) >= (lc, ld), indexed X(X+1)/2 + Y over
 * pair classes X = la(la+1)/2 + lb (Section 5: quartets grouped by
 * angular momentum).  mjk_class_l writes la, lb, lc, ld of class q. */
int mjk_num_classes(void);
int mjk_class_l(int32_t q, int32_t *l4);

/* Message of the last failure on the calling thread ("" if none). */
const char *mjk_last_error(void);

/* Message of the last failed call made with `ctx` or one of its plans or
 * batches, on any thread ("" if none).  The pointer stays valid on the
 * calling thread until its next call of this function. */
const char *mjk_ctx_last_error(mjk_ctx *ctx);

/* Context on HIP device `device` (must be gfx950).  Returns MJK_ERR_NO_DEVICE
 * when no such device exists. */
int mjk_ctx_create(int device, mjk_ctx **out);
void mjk_ctx_destroy(mjk_ctx *ctx);

/* Number of Cartesian basis functions of `basis` (host-only, no device). */
int mjk_nbf(const mjk_basis *basis, int64_t *nbf);

/* Validate the basis and options, copy them, and report the device
 * workspace the plan needs (bytes, 256-byte aligned start required).
 * Host-only: no device memory is touched. */
int mjk_plan_create(mjk_ctx *ctx, const mjk_basis *basis, const mjk_jk_opts *opts, mjk_plan **out,
                    size_t *workspace_bytes);

/* Bind the caller's device workspace and build the tables in it, on
 * `stream`: shell-pair and primitive-pair tables, Schwarz factors, the
 * class-sorted pair order and the quartet work lists (Section 5: pairs
 * sorted by angular momentum and tiled within a class; quartet blocks are
 * formed from pair tiles).  Synchronizes `stream` once (the Schwarz factors
 * come back to the host for the sort).  The work lists are built on up to
 * 16 host threads (fewer if OMP_NUM_THREADS says so), one bin pair at a
 * time per thread; their layout does not depend on the thread count.  The
 * workspace must stay allocated and untouched until mjk_plan_destroy or the
 * next bind. */
int mjk_plan_bind(mjk_plan *plan, void *workspace, size_t bytes, void *stream);

/* J and K for density D (nbf x nbf, symmetric), both overwritten.
 * D, J, K: device float64, row-major, distinct buffers.  Asynchronous on
 * `stream`.  With MJK_FLAG_CHECK in the plan's flags, D is copied to the
 * host and checked first (finite, symmetric to 1e-12 max|D|). */
int mjk_build_jk(mjk_plan *plan, const double *D, double *J, double *K, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): J and K as
 * mjk_build_jk computes them, but the persistent kernels' work counters and
 * the split classes' staging slots live in the library's static device
 * scratch (256 MiB per device, held from the first mjk_ctx_create on that
 * device until the process ends) instead of the plan's workspace.  The call
 * allocates nothing.  Any bound single plan may use it; a plan created with
 * MJK_FLAG_NO_STAGING (whose workspace lacks those regions) must.  A plan
 * whose split classes need a staging slot larger than the scratch gets
 * MJK_ERR_UNSUPPORTED; otherwise as many slots as fit are used (a launch
 * then has at most that many blocks).  All calls on one device share its
 * scratch: calls that overlap in time on one device (different streams, or
 * other threads) race and give wrong results; calls ordered on one stream do
 * not.  No per-class timing.  Asynchronous on `stream`. */
int mjk_build_jk_static(mjk_plan *plan, const double *D, double *J, double *K, void *stream);

/* E2 = 1/2 Tr(DJ) - 1/4 Tr(DK), the two-electron energy of a closed-shell
 * density D with its J and K (Section 2.1's Fock build: E2 is the energy
 * whose derivative with respect to D is J - K/2).  D, J, K: device float64
 * nbf x nbf; e2: one device float64, overwritten.  Asynchronous. */
int mjk_e2(mjk_plan *plan, const double *D, const double *J, const double *K, double *e2, void *stream);

/* Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt, m = 0..mmax, by the
 * device routine of the class kernels (Section 2.2: the recurrences start
 * from an analytic [00|00], which is a prefactor times F_m(T)).
 * T: device float64, n values (finite, >= 0; any other value gives NaN
 * rows).  F: device float64, n x (mmax + 1), row-major, overwritten.
 * mmax in 0..13 (MJK_ERR_UNSUPPORTED otherwise).  Asynchronous on `stream`. */
int mjk_boys(mjk_ctx *ctx, int32_t mmax, const double *T, int64_t n, double *F, void *stream);

/* Nuclear gradient of E2 at fixed D: grad[3*atom + i] = dE2/dR_{atom,i},
 * device float64 natom x 3, overwritten.  The basis functions move with
 * their atoms; d(ab|cd)/dA_i = 2 alpha (a+1_i b|cd) - a_i (a-1_i b|cd) on
 * three centres of every kept unique quartet, the fourth by translational
 * invariance, contracted with 4 D_ab D_cd - D_ac D_bd - D_ad D_bc.  Every
 * kept quartet is evaluated in FP64 (fp32_tau does not apply).  The plan
 * must have been created with MJK_FLAG_GRAD (else MJK_ERR_STATE); natom is
 * limited to 1024 (MJK_ERR_UNSUPPORTED).  Asynchronous on `stream`; with
 * timing enabled the per-class events cover this call's launches. */
int mjk_grad_e2(mjk_plan *plan, const double *D, double *grad, void *stream);

/* Backward of E2 = 1/2 Tr(DJ) - 1/4 Tr(DK) for automatic differentiation,
 * scaled by the upstream gradient: gout is one device float64 (dL/dE2), or
 * NULL for 1.
 *   gD (nbf x nbf, device float64, overwritten; NULL to skip):
 *       gout * (J - K/2), the derivative with respect to the entries of a
 *       symmetric D taken as independent (J and K are linear in D);
 *       needs J and K of that D (mjk_build_jk); must not alias them.
 *   gR (natom x 3, device float64, overwritten; NULL to skip):
 *       gout * dE2/dR at fixed D, as mjk_grad_e2 (MJK_FLAG_GRAD plans).
 * Asynchronous on `stream`. */
int mjk_e2_backward(mjk_plan *plan, const double *D, const double *J, const double *K, const double *gout,
                    double *gD, double *gR, void *stream);

/* Bins of shell pairs by primitive-pair count K_A K_B ("K-buckets": 1, 2-4,
 * 5-9, 10-16, 17-25, 26-36), inside each angular-momentum class. */
int mjk_num_kbuckets(void);

/* Work per lane (Section 7, Algorithm 2's workload): quartets per lane
 * (1, 2, 4, 8 or 16), i.e. a wave takes one bra pair and 64 * qpl of its
 * kets.  Either one value per class (n = mjk_num_classes(), qpl[q]) or one
 * per class and bra K-bucket (n = mjk_num_classes() * mjk_num_kbuckets(),
 * qpl[q * mjk_num_kbuckets() + k]).  Default 1.  Rebuilds the plan's work
 * lists (host, then a synchronous upload; waits for the device to be idle
 * first).  Results change only in summation order. */
int mjk_plan_set_tiles(mjk_plan *plan, const int32_t *qpl, int32_t n);

/* Explicit contracted ERI blocks (Eq. 2) for nq shell quartets.
 * quartets: host int32, nq x 4 shell indices (A, B, C, D) in any order.
 * out: device float64; quartet q occupies na*nb*nc*nd values, row-major over
 * (a, b, c, d) in the caller's shell order, blocks back to back in request
 * order; out_len must equal the total.  No screening is applied; the plan's
 * fp32_tau is: a quartet with Q_AB Q_CD < fp32_tau runs its vertical
 * recurrence and contraction in FP32 as in mjk_build_jk, so that the FP32
 * error of single integrals can be measured. */
int mjk_eri_class(mjk_plan *plan, const int32_t *quartets, int64_t nq, double *out, int64_t out_len,
                  void *stream);

/* Density-weighted screening for incremental Fock builds (the paper's
 * related work limits the integrals recomputed per SCF iteration; J and K are
 * linear in D, so J(D_n) = J(D_{n-1}) + J(D_n - D_{n-1})).  dD: device
 * float64 nbf x nbf (the density change), read during the call only.  The
 * plan's work lists are rebuilt so that, on top of the Schwarz screen, a
 * unique quartet (AB|CD) is skipped when
 *     Q_AB Q_CD max(w_A, w_B, w_C, w_D') < tau   (tau >= 0, finite),
 * with w_X the largest |dD| in the rows of shell X and w_D' the largest w
 * over the second shells of the kets of C's run (a bound on every D block a
 * quartet's J and K updates read: each contribution is at most
 * |(ab|cd)| max |dD| over those blocks).  dD = NULL restores the plain lists.
 * The screen stays in force for every later mjk_build_jk of the plan.
 * Synchronizes the device (host rebuild of the lists on the threads
 * mjk_plan_bind uses, then an upload).  MJK_ERR_UNSUPPORTED if host memory
 * runs out for the lists (mjk_plan_bind alike). */
int mjk_plan_set_density_screen(mjk_plan *plan, const double *dD, double tau, void *stream);

/* One-electron matrices of the SCF iteration (Section 2.1: the Fock matrix
 * is the one-electron Hamiltonian T + V plus the two-electron part J - K/2):
 *   S_mn = <m|n>,  T_mn = <m| -1/2 nabla^2 |n>,
 *   V_mn = sum_C -Z_C <m| 1/|r - R_C| |n>  (point charges at the atom centres).
 * S, T, V: device float64 nbf x nbf row-major, overwritten; each may be NULL
 * (skipped); non-null ones must be distinct.  Z: device float64, natom
 * charges (finite; the call does not read them on the host).  enuc: one
 * device float64, sum_{A<B} Z_A Z_B / |R_A - R_B|, or NULL.  Needs a bound
 * single plan (MJK_ERR_STATE otherwise).  Asynchronous on `stream`. */
int mjk_one_electron(mjk_plan *plan, const double *Z, double *S, double *T, double *V, double *enuc,
                     void *stream);

/* Schwarz factors Q[A][B] (host float64, nshell x nshell, symmetric) as
 * used by the plan.  Synchronous. */
int mjk_schwarz(mjk_plan *plan, double *Q_host);

/* Plan statistics (host, synchronous, no device work). */
int mjk_plan_stats_get(const mjk_plan *plan, mjk_plan_stats *stats);

/* Per-class kernel timing, for measurement tools.  With timing enabled,
 * mjk_build_jk records a HIP event pair on `stream` around every class
 * launch.  After that stream has completed, mjk_plan_timings sums, per
 * quartet class (la lb | lc ld), the milliseconds and launches of the last
 * mjk_build_jk, and the algorithmic work they covered: primitive quartets,
 * shell quartets and floating-point operations (per primitive quartet:
 * geometry, Boys function, vertical recurrence and accumulation; per shell
 * quartet: horizontal recurrence and digestion, 12 flops per integral).
 * out: host array of cap records; *n receives the number of classes with
 * work (at most cap are written).  Synchronizes nothing itself; returns
 * MJK_ERR_STATE if timing was off during the last build.  After
 * mjk_grad_e2 the records describe that call (flops: its algorithmic work,
 * all shifted classes of each class). */
typedef struct mjk_class_timing {
    int32_t la, lb, lc, ld;
    int32_t nlaunch;
    double ms;
    int64_t nquartet;
    int64_t nprim_quartet;
    double flops;
} mjk_class_timing;

int mjk_plan_set_timing(mjk_plan *plan, int enable);
int mjk_plan_timings(mjk_plan *plan, mjk_class_timing *out, int32_t cap, int32_t *n);

void mjk_plan_destroy(mjk_plan *plan);

/* ---- Batches: many molecules of uneven size in one launch per class ----
 * Section 5's blocks of every molecule, concatenated: each launch takes the
 * work of one quartet class (at one precision) for all molecules, costliest
 * segments first, and persistent waves pull work items from an atomic
 * counter.  Molecule m's D, J, K are nbf_m x nbf_m row-major blocks packed
 * back to back in one device buffer, at the element offsets given by
 * mjk_batch_offsets (nmol + 1 values, the last = total length).  The
 * results equal those of separate plans up to summation order.
 *
 * mjk_batch_create: validates every molecule (as mjk_plan_create) with the
 *   same options (no MJK_FLAG_GRAD); reports the workspace bytes.
 * mjk_batch_bind: builds every molecule's tables in the workspace
 *   (synchronizes `stream` once per molecule).
 * mjk_batch_build_jk: J and K of every molecule, overwritten; asynchronous.
 * mjk_batch_set_tiles: quartets per lane, as mjk_plan_set_tiles.
 * mjk_batch_autotune: Algorithm 2 on this batch.  qpl (in/out, n values)
 *   is a table per class (n = mjk_num_classes()) or per class and bra
 *   K-bucket (n = classes x mjk_num_kbuckets()); entries 0 are tuned (they
 *   start at one quartet per lane), the others stay as given.  Each sweep
 *   times an entry's class alone (shortest of `reps` launches), doubles the
 *   entry's workload (Combine), times it again and keeps the change if
 *   faster, else halves it back (Revert) and retires the entry; sweeps repeat
 *   while any entry improved.  The result is written back to qpl and left
 *   active.  Synchronous; J and K hold no meaningful values afterwards.
 * mjk_batch_set_stamps: record per-molecule wall-clock stamps (first work
 *   item started, last work item finished) during builds;
 *   mjk_batch_mol_times converts those of the last build to milliseconds
 *   since the earliest start, ms[2m], ms[2m+1] (synchronous).
 * mjk_batch_set_timing / mjk_batch_timings: per-class event timing, as for
 *   plans.
 * mjk_batch_stats: totals over molecules; nq_per_mol (optional, nmol values)
 *   receives each molecule's kept quartets. */
typedef struct mjk_batch mjk_batch;
int mjk_batch_create(mjk_ctx *ctx, int32_t nmol, const mjk_basis *mols, const mjk_jk_opts *opts, mjk_batch **out,
                     size_t *workspace_bytes);
int mjk_batch_bind(mjk_batch *batch, void *workspace, size_t bytes, void *stream);
int mjk_batch_offsets(const mjk_batch *batch, int64_t *mat_off);
int mjk_batch_build_jk(mjk_batch *batch, const double *D, double *J, double *K, void *stream);
int mjk_batch_set_tiles(mjk_batch *batch, const int32_t *qpl, int32_t n);
int mjk_batch_autotune(mjk_batch *batch, const double *D, double *J, double *K, int32_t reps, int32_t *qpl,
                       int32_t n, void *stream);
int mjk_batch_set_stamps(mjk_batch *batch, int enable);
int mjk_batch_mol_times(mjk_batch *batch, double *ms);
int mjk_batch_set_timing(mjk_batch *batch, int enable);
int mjk_batch_timings(mjk_batch *batch, mjk_class_timing *out, int32_t cap, int32_t *n);
int mjk_batch_stats(const mjk_batch *batch, mjk_plan_stats *total, int64_t *nq_per_mol);
void mjk_batch_destroy(mjk_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* MJK_H */
