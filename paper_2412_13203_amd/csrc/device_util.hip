// device_util.hip -- the small non-class kernels: primitive-pair table,
// fill, in-place symmetrization, E2 and its backward, and the Boys function
// evaluated on its own.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mjk_types.hpp"

namespace mjk {

struct ShellArrays {
    const double *xyz;       // natom x 3
    const int32_t *atom;     // nshell
    const int32_t *prim_off; // nshell
    const int32_t *nprim;    // nshell
    const double *exps;
    const double *coefs;
};

// One primitive pair per thread: p, 1/(2p), P, P - A and the folded
// prefactor K = sqrt(2) pi^{5/4} c_a c_b exp(-ab/p |AB|^2) / p  (Eq. 2's
// coefficients and the Gaussian product of the two primitives).
__global__ __launch_bounds__(256) void k_pair_table(const ShellPairD *__restrict__ pairs, int npair,
                                                    ShellArrays sh, PrimPairD *__restrict__ out, int nprim_pair)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nprim_pair) return;
    int lo = 0, hi = npair;  // pairs[lo].prim_off <= t < pairs[lo+1].prim_off
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pairs[mid].prim_off <= t)
            lo = mid;
        else
            hi = mid;
    }
    const ShellPairD pr = pairs[lo];
    const int local = t - pr.prim_off;
    // nprim = K_A * K_B, A-major
    const int KB = sh.nprim[pr.B];
    const int i = local / KB, j = local % KB;
    const int ia = sh.prim_off[pr.A] + i, jb = sh.prim_off[pr.B] + j;
    const double al = sh.exps[ia], be = sh.exps[jb];
    const double *A = sh.xyz + 3 * sh.atom[pr.A];
    const double *B = sh.xyz + 3 * sh.atom[pr.B];
    const double p = al + be;
    const double ip = 1.0 / p;
    PrimPairD o;
    o.p = p;
    o.oo2p = 0.5 * ip;
    double ab2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        const double Px = (al * A[x] + be * B[x]) * ip;
        o.P[x] = Px;
        o.PA[x] = Px - A[x];
        ab2 += (A[x] - B[x]) * (A[x] - B[x]);
    }
    const double c0 = 0x1.7a8ed27904870p+2;  // sqrt(2) pi^(5/4) = 5.914967172795613
    o.K = c0 * sh.coefs[ia] * sh.coefs[jb] * exp(-al * be * ip * ab2) * ip;
    o.alpha = al;
    out[t] = o;
}

__global__ __launch_bounds__(256) void k_fill(double *__restrict__ x, int64_t n, double v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

// M <- M + M^T in place; the thread of (i, j), i < j, owns both elements.
__global__ __launch_bounds__(256) void k_symmetrize(double *__restrict__ M, int n)
{
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= n || j >= n || i > j) return;
    if (i == j) {
        M[(size_t)i * n + i] *= 2.0;
    } else {
        const double s = M[(size_t)i * n + j] + M[(size_t)j * n + i];
        M[(size_t)i * n + j] = s;
        M[(size_t)j * n + i] = s;
    }
}

// E2 = sum_ij D_ij (J_ij / 2 - K_ij / 4): one block, fixed summation order
// (strided partial sums, then a tree in LDS), so repeated calls agree bitwise.
__global__ __launch_bounds__(1024) void k_e2(const double *__restrict__ D, const double *__restrict__ J,
                                             const double *__restrict__ K, int64_t n2, double *__restrict__ e2)
{
    __shared__ double part[1024];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < n2; t += 1024) s += D[t] * (0.5 * J[t] - 0.25 * K[t]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 512; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *e2 = part[0];
}

int launch_e2(const double *D, const double *J, const double *K, int n, double *e2, hipStream_t s)
{
    if (n <= 0) return -1;
    hipLaunchKernelGGL(k_e2, dim3(1), dim3(1024), 0, s, D, J, K, (int64_t)n * n, e2);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pair_table(const ShellPairD *pairs, int npair, const double *xyz, const int32_t *atom,
                      const int32_t *prim_off, const int32_t *nprim, const double *exps, const double *coefs,
                      PrimPairD *out, int nprim_pair, hipStream_t s)
{
    if (nprim_pair <= 0) return 0;
    ShellArrays sh{xyz, atom, prim_off, nprim, exps, coefs};
    hipLaunchKernelGGL(k_pair_table, dim3((nprim_pair + 255) / 256), dim3(256), 0, s, pairs, npair, sh, out,
                       nprim_pair);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill(double *x, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ x, int64_t n, uint32_t v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

// per molecule: [first start, last end] = [max, 0] before a build
__global__ __launch_bounds__(256) void k_stamp_init(unsigned long long *__restrict__ x, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        x[2 * t] = ~0ull;
        x[2 * t + 1] = 0ull;
    }
}

int launch_fill_u32(uint32_t *x, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_stamp_init(unsigned long long *x, int n, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_stamp_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_symmetrize(double *M, int n, hipStream_t s)
{
    if (n <= 0) return 0;
    const unsigned g = (unsigned)((n + 15) / 16);
    hipLaunchKernelGGL(k_symmetrize, dim3(g, g), dim3(256), 0, s, M, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// dE2/dD = g (J - K/2): E2 = 1/2 Tr(DJ) - 1/4 Tr(DK) with J and K linear in
// D, so the derivative with respect to the entries of a symmetric D (taken
// as independent) is J - K/2; g is the upstream gradient (device scalar,
// NULL = 1).
__global__ __launch_bounds__(256) void k_e2_grad_D(const double *__restrict__ J, const double *__restrict__ K,
                                                   const double *__restrict__ g, double *__restrict__ out, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double s = g ? *g : 1.0;
    out[t] = s * (J[t] - 0.5 * K[t]);
}

__global__ __launch_bounds__(256) void k_scale(double *__restrict__ x, int64_t n, const double *__restrict__ g)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] *= *g;
}

int launch_e2_grad_D(const double *J, const double *K, const double *g, double *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_e2_grad_D, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, J, K, g, out, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_scale(double *x, int64_t n, const double *g, hipStream_t s)
{
    if (n <= 0 || !g) return 0;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, g);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// F_m(T), m = 0..M, by the same device routine the class kernels call with
// L = M (Section 2.2's analytic [00|00]); one argument per thread.  T must be
// finite and >= 0: any other argument gives NaN rather than a table read.
template <int M>
__global__ __launch_bounds__(256) void k_boys(const double *__restrict__ T, int64_t n, double *__restrict__ F)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double x = T[t];
    double f[M + 1];
    if (x >= 0.0 && x <= 1.0e300) {
        boys_fm<M>(x, f);
    } else {
#pragma unroll
        for (int m = 0; m <= M; ++m) f[m] = __builtin_nan("");
    }
#pragma unroll
    for (int m = 0; m <= M; ++m) F[t * (M + 1) + m] = f[m];
}

template <int M>
int launch_boys_m(const double *T, int64_t n, double *F, hipStream_t s)
{
    hipLaunchKernelGGL(k_boys<M>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, n, F);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int M>
int launch_boys_upto(int mmax, const double *T, int64_t n, double *F, hipStream_t s)
{
    if (mmax == M) return launch_boys_m<M>(T, n, F, s);
    if constexpr (M > 0)
        return launch_boys_upto<M - 1>(mmax, T, n, F, s);
    else
        return -1;
}

// out[r] = max_c |M[r][c]|, one block per row (n x n row-major)
__global__ __launch_bounds__(256) void k_rowmax_abs(const double *__restrict__ M, int n, double *__restrict__ out)
{
    __shared__ double part[256];
    const double *row = M + (size_t)blockIdx.x * n;
    double m = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) {
        const double v = fabs(row[c]);
        m = v == v ? fmax(m, v) : __builtin_huge_val();  // a NaN reads as infinite
    }
    part[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

int launch_rowmax_abs(const double *M, int n, double *out, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_rowmax_abs, dim3((unsigned)n), dim3(256), 0, s, M, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int boys_lmax() { return MJK_BOYS_LMAX; }

int launch_boys(int mmax, const double *T, int64_t n, double *F, hipStream_t s)
{
    if (n <= 0) return 0;
    if (mmax < 0 || mmax > MJK_BOYS_LMAX) return -1;
    return launch_boys_upto<MJK_BOYS_LMAX>(mmax, T, n, F, s);
}

}  // namespace mjk
