// one_electron.hip -- overlap, kinetic-energy and nuclear-attraction
// integrals over contracted Cartesian shells, and the repulsion of the point
// nuclei.  With J and K they make the Fock matrix that the SCF iteration
// rebuilds from the density at every step (Section 2.1: the Fock matrix is
// the one-electron Hamiltonian plus the two-electron part).
//
// Route: Obara-Saika.  Per primitive pair (exponents a on A, b on B,
// p = a + b, P = (aA + bB)/p, E_AB = c_a c_b exp(-ab/p |AB|^2)):
//   overlap and kinetic energy factor into 1-D integrals per axis, built by
//     s_{i+1,j} = X_PA s_ij + (i s_{i-1,j} + j s_{i,j-1}) / 2p,
//     s_{i,j+1} = X_PB s_ij + (i s_{i-1,j} + j s_{i,j-1}) / 2p,   s_00 = 1,
//     t_{i+1,j} = X_PA t_ij + (i t_{i-1,j} + j t_{i,j-1}) / 2p + (b/p)(2a s_{i+1,j} - i s_{i-1,j}),
//     t_{i,j+1} = X_PB t_ij + (i t_{i-1,j} + j t_{i,j-1}) / 2p + (a/p)(2b s_{i,j+1} - j s_{i,j-1}),
//     t_00 = a - 2a^2 (X_PA^2 + 1/2p),
//   S = E_AB (pi/p)^{3/2} s^x s^y s^z,
//   T = E_AB (pi/p)^{3/2} (t^x s^y s^z + s^x t^y s^z + s^x s^y t^z);
//   nuclear attraction to a charge Z at C by the vertical recurrence on the
//   first centre (U = p |PC|^2, F_m the Boys function)
//     [e + 1_i]^(m) = X_PA,i [e]^(m) - X_PC,i [e]^(m+1)
//                     + e_i / 2p ([e - 1_i]^(m) - [e - 1_i]^(m+1)),
//     [0]^(m) = -Z 2 pi / p E_AB F_m(U),
//   summed over primitive pairs and nuclei for la <= |e| <= la + lb, then
//   moved to the second centre through the binomial form of the horizontal
//   recurrence (x - B = (x - A) + (A - B) on each axis):
//     (a|V|b) = sum_{k <= b} prod_i C(b_i, k_i) (A - B)_i^{b_i - k_i} [a + k].
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mjk_types.hpp"

namespace mjk {

namespace {

constexpr double kPi = 3.14159265358979323846;
// sqrt(2) pi^{5/4}: the primitive-pair table stores K = this * E_AB / p
constexpr double kPairK = 0x1.7a8ed27904870p+2;

// index of the Cartesian component (x, y, z), x + y + z = l, in lexicographic
// order (xx, xy, xz, yy, yz, zz for l = 2)
__host__ __device__ constexpr int comp_index(int l, int x, int z) { return (l - x) * (l - x + 1) / 2 + z; }

// exponents of component c of level l
__host__ __device__ constexpr void comp_exps(int l, int c, int &x, int &y, int &z)
{
    int k = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j, ++k)
            if (k == c) {
                x = i;
                y = j;
                z = l - i - j;
                return;
            }
    x = y = z = 0;
}

// first component of level l in a table holding levels 0..l-1 before it
__host__ __device__ constexpr int level_off(int l) { return l * (l + 1) * (l + 2) / 6; }

// 1-D overlap and kinetic tables s[i][j], t[i][j], i <= NI, j <= NJ
template <int NI, int NJ>
__device__ __forceinline__ void one_d(double PA, double PB, double oo2p, double a, double b, double ip,
                                      double (&s)[NI + 1][NJ + 1], double (&t)[NI + 1][NJ + 1])
{
    s[0][0] = 1.0;
    t[0][0] = a - 2.0 * a * a * (PA * PA + oo2p);
    const double bp = b * ip, ap = a * ip;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const double sm = i ? s[i - 1][0] : 0.0, tm = i ? t[i - 1][0] : 0.0;
        s[i + 1][0] = PA * s[i][0] + oo2p * i * sm;
        t[i + 1][0] = PA * t[i][0] + oo2p * i * tm + bp * (2.0 * a * s[i + 1][0] - i * sm);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int i = 0; i <= NI; ++i) {
            const double si = i ? s[i - 1][j] : 0.0, ti = i ? t[i - 1][j] : 0.0;
            const double sj = j ? s[i][j - 1] : 0.0, tj = j ? t[i][j - 1] : 0.0;
            s[i][j + 1] = PB * s[i][j] + oo2p * (i * si + j * sj);
            t[i][j + 1] = PB * t[i][j] + oo2p * (i * ti + j * tj) + ap * (2.0 * b * s[i][j + 1] - j * sj);
        }
    }
}

// Nuclear-attraction vertical recurrence of one (primitive pair, nucleus):
// th holds [e]^(m) for |e| <= L, level by level, m = 0..L-|e| per component
// (m-major inside a level); acc[e - level_off(LA)] += [e]^(0) for |e| >= LA.
template <int LA, int L>
__device__ __forceinline__ void vrr_nuc(const double (&F)[L + 1], double pre, const double (&PA)[3],
                                        const double (&PC)[3], double oo2p, double *acc)
{
    // [e]^(m) of the current and the two previous levels
    double cur[ncart(L)][L + 1], prev[ncart(L)][L + 1], prev2[ncart(L)][L + 1];
#pragma unroll
    for (int m = 0; m <= L; ++m) cur[0][m] = pre * F[m];
    if (LA == 0) acc[0] += cur[0][0];
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        // level l - 2 moves to prev2, level l - 1 to prev
        if (l >= 2) {
#pragma unroll
            for (int c = 0; c < ncart(l - 2); ++c)
#pragma unroll
                for (int m = 0; m <= L - l + 2; ++m) prev2[c][m] = prev[c][m];
        }
#pragma unroll
        for (int c = 0; c < ncart(l - 1); ++c)
#pragma unroll
            for (int m = 0; m <= L - l + 1; ++m) prev[c][m] = cur[c][m];
#pragma unroll
        for (int c = 0; c < ncart(l); ++c) {
            int x = 0, y = 0, z = 0;
            comp_exps(l, c, x, y, z);
            // step down along the first axis with a non-zero exponent
            const int i = x ? 0 : (y ? 1 : 2);
            const int ex = x - (i == 0), ey = y - (i == 1), ez = z - (i == 2);
            const int e_i = i == 0 ? ex : (i == 1 ? ey : ez);
            const int c1 = comp_index(l - 1, ex, ez);
            const int c2 = e_i ? comp_index(l - 2, ex - (i == 0), ez - (i == 2)) : 0;
#pragma unroll
            for (int m = 0; m <= L - l; ++m) {
                double v = PA[i] * prev[c1][m] - PC[i] * prev[c1][m + 1];
                if (e_i) v += (e_i * oo2p) * (prev2[c2][m] - prev2[c2][m + 1]);
                cur[c][m] = v;
            }
            if (l >= LA) acc[level_off(l) - level_off(LA) + c] += cur[c][0];
        }
    }
}

struct OneELaunch {
    const ShellPairD *pairs;  // natural pair table
    const PrimPairD *prims;
    const int32_t *idx;       // natural pair indices of one pair class
    int32_t n;
    const double *xyz;        // natom x 3
    const double *Z;          // natom
    int32_t natom;
    int32_t nbf;
    double *S, *T, *V;        // nbf x nbf; any may be null
};

// One wave per shell pair of class (LA, LB), LA >= LB.
template <int LA, int LB>
__global__ __launch_bounds__(64) void k_one_electron(OneELaunch a)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), L = LA + LB;
    constexpr int NE = level_off(L + 1) - level_off(LA);
    __shared__ double sE[NE];
    const int lane = threadIdx.x;
    const ShellPairD sp = a.pairs[a.idx[blockIdx.x]];
    const PrimPairD *pr = a.prims + sp.prim_off;
    const int np = sp.nprim;
    const int n = a.nbf;

    // overlap and kinetic energy: one component pair per lane
    if (a.S || a.T) {
        for (int c = lane; c < NA * NB; c += 64) {
            const int ia = c / NB, ib = c % NB;
            if (sp.same && ia < ib) continue;  // the (ib, ia) lane writes both
            int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
            comp_exps(LA, ia, ax, ay, az);
            comp_exps(LB, ib, bx, by, bz);
            double sv = 0.0, tv = 0.0;
            for (int k = 0; k < np; ++k) {
                const PrimPairD q = pr[k];
                const double ip = 2.0 * q.oo2p;
                const double al = q.alpha, be = q.p - al;
                const double pre = q.K * q.p * (1.0 / kPairK) * kPi * ip * sqrt(kPi * ip);
                double s[3], t[3];
                const int ea[3] = {ax, ay, az}, eb[3] = {bx, by, bz};
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    double st[LA + 1][LB + 1], tt[LA + 1][LB + 1];
                    one_d<LA, LB>(q.PA[x], q.PA[x] + sp.AB[x], q.oo2p, al, be, ip, st, tt);
                    // select (ea[x], eb[x]) without dynamic indexing of the tables
                    double sv1 = 0.0, tv1 = 0.0;
#pragma unroll
                    for (int i = 0; i <= LA; ++i)
#pragma unroll
                        for (int j = 0; j <= LB; ++j)
                            if (i == ea[x] && j == eb[x]) {
                                sv1 = st[i][j];
                                tv1 = tt[i][j];
                            }
                    s[x] = sv1;
                    t[x] = tv1;
                }
                sv += pre * s[0] * s[1] * s[2];
                tv += pre * (t[0] * s[1] * s[2] + s[0] * t[1] * s[2] + s[0] * s[1] * t[2]);
            }
            const int r = sp.ao_a + ia, col = sp.ao_b + ib;
            if (a.S) {
                a.S[(size_t)r * n + col] = sv;
                a.S[(size_t)col * n + r] = sv;
            }
            if (a.T) {
                a.T[(size_t)r * n + col] = tv;
                a.T[(size_t)col * n + r] = tv;
            }
        }
    }
    if (!a.V) return;

    // nuclear attraction: (primitive pair, nucleus) items over the lanes
    double acc[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] = 0.0;
    const int nitem = np * a.natom;
    for (int it = lane; it < nitem; it += 64) {
        const int k = it / a.natom, C = it - k * a.natom;
        const double Zc = a.Z[C];
        if (Zc == 0.0) continue;
        const PrimPairD q = pr[k];
        const double PA[3] = {q.PA[0], q.PA[1], q.PA[2]};
        const double PC[3] = {q.P[0] - a.xyz[3 * C], q.P[1] - a.xyz[3 * C + 1], q.P[2] - a.xyz[3 * C + 2]};
        const double ip = 2.0 * q.oo2p;
        const double U = q.p * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
        double F[L + 1];
        boys_fm<L>(U, F);
        const double pre = -Zc * 2.0 * kPi * ip * q.K * q.p * (1.0 / kPairK);
        vrr_nuc<LA, L>(F, pre, PA, PC, q.oo2p, acc);
    }
    // sum the accumulators over the wave
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        double v = acc[e];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sE[e] = v;
    }
    __syncthreads();
    for (int c = lane; c < NA * NB; c += 64) {
        const int ia = c / NB, ib = c % NB;
        if (sp.same && ia < ib) continue;
        int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
        comp_exps(LA, ia, ax, ay, az);
        comp_exps(LB, ib, bx, by, bz);
        double v = 0.0;
        // binomial horizontal recurrence over k <= b
        for (int kx = 0; kx <= bx; ++kx)
            for (int ky = 0; ky <= by; ++ky)
                for (int kz = 0; kz <= bz; ++kz) {
                    double cf = 1.0;
                    // C(b_i, k_i) (A - B)_i^{b_i - k_i}
                    const int kk[3] = {kx, ky, kz}, bb[3] = {bx, by, bz};
                    for (int x = 0; x < 3; ++x) {
                        double binom = 1.0;
                        for (int u = 0; u < kk[x]; ++u) binom = binom * (bb[x] - u) / (u + 1);
                        double pw = 1.0;
                        for (int u = 0; u < bb[x] - kk[x]; ++u) pw *= sp.AB[x];
                        cf *= binom * pw;
                    }
                    const int le = LA + kx + ky + kz;
                    v += cf * sE[level_off(le) - level_off(LA) + comp_index(le, ax + kx, az + kz)];
                }
        const int r = sp.ao_a + ia, col = sp.ao_b + ib;
        a.V[(size_t)r * n + col] = v;
        a.V[(size_t)col * n + r] = v;
    }
}

template <int LA, int LB>
int launch_one_e_class(const OneELaunch &a, hipStream_t s)
{
    if (a.n <= 0) return 0;
    hipLaunchKernelGGL((k_one_electron<LA, LB>), dim3((unsigned)a.n), dim3(64), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// sum_{A<B} Z_A Z_B / |R_A - R_B| by one block in a fixed order; centres
// without charge add nothing (also where they coincide with an atom)
__global__ __launch_bounds__(256) void k_nuclear_repulsion(const double *__restrict__ xyz,
                                                           const double *__restrict__ Z, int natom,
                                                           double *__restrict__ out)
{
    __shared__ double part[256];
    double e = 0.0;
    for (int A = threadIdx.x; A < natom; A += 256)
        for (int B = 0; B < A; ++B) {
            if (Z[A] == 0.0 || Z[B] == 0.0) continue;
            const double dx = xyz[3 * A] - xyz[3 * B], dy = xyz[3 * A + 1] - xyz[3 * B + 1],
                         dz = xyz[3 * A + 2] - xyz[3 * B + 2];
            e += Z[A] * Z[B] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    part[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

}  // namespace

// S, T, V over every shell pair of the natural pair table (class by class)
// and, when enuc is not null, the nuclear repulsion.
int launch_one_electron(const ShellPairD *pairs, const PrimPairD *prims, const int32_t *cls_idx,
                        const int32_t *cls_off, int lmax, const double *xyz, const double *Z, int natom, int nbf,
                        double *S, double *T, double *V, double *enuc, hipStream_t s)
{
    for (int la = 0; la <= lmax; ++la)
        for (int lb = 0; lb <= la; ++lb) {
            const int c = la * (la + 1) / 2 + lb;
            OneELaunch a{pairs, prims, cls_idx + cls_off[c], cls_off[c + 1] - cls_off[c], xyz, Z, natom, nbf,
                         S, T, V};
            int rc = 0;
            switch (c) {
            case 0: rc = launch_one_e_class<0, 0>(a, s); break;
            case 1: rc = launch_one_e_class<1, 0>(a, s); break;
            case 2: rc = launch_one_e_class<1, 1>(a, s); break;
            case 3: rc = launch_one_e_class<2, 0>(a, s); break;
            case 4: rc = launch_one_e_class<2, 1>(a, s); break;
            case 5: rc = launch_one_e_class<2, 2>(a, s); break;
            case 6: rc = launch_one_e_class<3, 0>(a, s); break;
            case 7: rc = launch_one_e_class<3, 1>(a, s); break;
            case 8: rc = launch_one_e_class<3, 2>(a, s); break;
            case 9: rc = launch_one_e_class<3, 3>(a, s); break;
            default: rc = -1;
            }
            if (rc) return rc;
        }
    if (enuc) {
        hipLaunchKernelGGL(k_nuclear_repulsion, dim3(1), dim3(256), 0, s, xyz, Z, natom, enuc);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace mjk
