// Contact angle of a droplet from the density fields (FP64), for the
// single lattice and for every run of a batch (arXiv 2505.22256, Sec. 3.2;
// the paper does not say how it measures the angle).  Reads the rho1 / rho2
// fields that the fields pass of the step kernel writes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

// ---------------------------------------------------------------------------
// Contact angle (FP64): interface points of rho^e = 0 along links, algebraic
// circle fit, Gauss-Newton refinement, angle with the wall.
// ---------------------------------------------------------------------------
struct WallDesc {
    int kind;
    double w0, w1, w2;
};

// ---------------------------------------------------------------------------
// Phase regions.  Fluid nodes split into rho^e > 0 and rho^e <= 0; regions
// are 4-connected along x and y links (not across periodic seams).  Only
// the interface between the largest region of each phase (the droplet and
// the fluid around it) is fitted, so pockets trapped under a droplet and
// satellite droplets do not bend the circle.  Union-find with the smaller
// index as the root: every region's root is its smallest node, which also
// breaks ties between equally large regions.  Grid: blockIdx.y = run,
// blockIdx.x strides over the run's nodes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool phase_positive(const double *r1, const double *r2, long long a)
{
    return (r1[a] - r2[a]) / (r1[a] + r2[a]) > 0.0;
}

static __global__ void __launch_bounds__(256)
k_cc_init(const int *__restrict__ dims, const long long *__restrict__ offs, const uint8_t *__restrict__ solid,
          int *__restrict__ par, int *__restrict__ cnt)
{
    const int run = blockIdx.y;
    const long long N = (long long)dims[2 * run] * dims[2 * run + 1], off = offs[run];
    for (long long a = (long long)blockIdx.x * 256 + threadIdx.x; a < N; a += (long long)gridDim.x * 256) {
        par[off + a] = solid[off + a] ? -1 : (int)a;
        cnt[off + a] = 0;
    }
}

// Root of x.  Loads are device-coherent because other lanes link roots
// concurrently; parents only ever point to smaller indices, so the walk ends.
__device__ __forceinline__ int cc_find(int *par, int x)
{
    for (;;) {
        const int p = __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x) return x;
        x = p;
    }
}

// Link the larger root under the smaller.  A failed compare-and-swap means
// another lane linked that root first; every retry follows a successful link
// elsewhere, so the loop ends.
__device__ __forceinline__ void cc_unite(int *par, int a, int b)
{
    for (;;) {
        const int ra = cc_find(par, a), rb = cc_find(par, b);
        if (ra == rb) return;
        const int hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
        if (atomicCAS(par + hi, hi, lo) == hi) return;
    }
}

static __global__ void __launch_bounds__(256)
k_cc_hook(const int *__restrict__ dims, const long long *__restrict__ offs, const double *__restrict__ rho1,
          const double *__restrict__ rho2, const uint8_t *__restrict__ solid, int *par_all)
{
    const int run = blockIdx.y, nx = dims[2 * run], ny = dims[2 * run + 1];
    const long long N = (long long)nx * ny, off = offs[run];
    const double *r1 = rho1 + off, *r2 = rho2 + off;
    const uint8_t *sd = solid + off;
    int *par = par_all + off;
    for (long long a = (long long)blockIdx.x * 256 + threadIdx.x; a < N; a += (long long)gridDim.x * 256) {
        if (sd[a]) continue;
        const int x = (int)(a % nx), y = (int)(a / nx);
        const bool pa = phase_positive(r1, r2, a);
        if (x + 1 < nx && !sd[a + 1] && phase_positive(r1, r2, a + 1) == pa) cc_unite(par, (int)a, (int)a + 1);
        if (y + 1 < ny && !sd[a + nx] && phase_positive(r1, r2, a + nx) == pa)
            cc_unite(par, (int)a, (int)(a + nx));
    }
}

// After hooking: par[a] <- root(a) for every fluid node, and region sizes.
static __global__ void __launch_bounds__(256)
k_cc_count(const int *__restrict__ dims, const long long *__restrict__ offs, const uint8_t *__restrict__ solid,
           int *par_all, int *cnt_all)
{
    const int run = blockIdx.y;
    const long long N = (long long)dims[2 * run] * dims[2 * run + 1], off = offs[run];
    int *par = par_all + off, *cnt = cnt_all + off;
    for (long long a = (long long)blockIdx.x * 256 + threadIdx.x; a < N; a += (long long)gridDim.x * 256) {
        if (solid[off + a]) continue;
        int r = (int)a;
        while (par[r] != r) r = par[r];
        par[a] = r;
        atomicAdd(cnt + r, 1);
    }
}

// One workgroup per run: best[2 run + phase] = root of the largest region of
// that phase (ties: the smaller root), -1 when the phase is absent.
static __global__ void __launch_bounds__(256)
k_cc_pick(const int *__restrict__ dims, const long long *__restrict__ offs, const double *__restrict__ rho1,
          const double *__restrict__ rho2, const uint8_t *__restrict__ solid, const int *__restrict__ par_all,
          const int *__restrict__ cnt_all, int *__restrict__ best)
{
    __shared__ unsigned long long sh[2][256];
    const int run = blockIdx.x, t = threadIdx.x;
    const long long N = (long long)dims[2 * run] * dims[2 * run + 1], off = offs[run];
    const int *par = par_all + off, *cnt = cnt_all + off;
    unsigned long long key[2] = {0ull, 0ull};
    for (long long a = t; a < N; a += 256) {
        if (solid[off + a] || par[a] != (int)a) continue;
        const int ph = phase_positive(rho1 + off, rho2 + off, a) ? 1 : 0;
        const unsigned long long k = ((unsigned long long)(unsigned)cnt[a] << 32) | (0xffffffffull - (unsigned long long)a);
        if (k > key[ph]) key[ph] = k;
    }
    sh[0][t] = key[0];
    sh[1][t] = key[1];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int q = 0; q < 2; ++q)
                if (sh[q][t + h] > sh[q][t]) sh[q][t] = sh[q][t + h];
        __syncthreads();
    }
    if (t < 2) {
        const unsigned long long k = sh[t][0];
        best[2 * run + t] = k ? (int)(0xffffffffull - (k & 0xffffffffull)) : -1;
    }
}

// Host side: label the phase regions of nruns runs (node counts up to
// max_nodes) and pick the largest of each phase; par and cnt hold one int
// per node at the runs' offsets, best two ints per run.
static inline hipError_t launch_phase_regions(hipStream_t st, const int *dims, const long long *offs, int nruns,
                                              long long max_nodes, const double *rho1, const double *rho2,
                                              const uint8_t *solid, int *par, int *cnt, int *best)
{
    long long bx = (max_nodes + 255) / 256;
    const long long cap = nruns > 1 ? 128 : 2048;
    if (bx > cap) bx = cap;
    if (bx < 1) bx = 1;
    const dim3 grid((unsigned)bx, (unsigned)nruns);
    hipLaunchKernelGGL(k_cc_init, grid, dim3(256), 0, st, dims, offs, solid, par, cnt);
    hipLaunchKernelGGL(k_cc_hook, grid, dim3(256), 0, st, dims, offs, rho1, rho2, solid, par);
    hipLaunchKernelGGL(k_cc_count, grid, dim3(256), 0, st, dims, offs, solid, par, cnt);
    hipLaunchKernelGGL(k_cc_pick, dim3((unsigned)nruns), dim3(256), 0, st, dims, offs, rho1, rho2, solid,
                       (const int *)par, (const int *)cnt, best);
    return hipGetLastError();
}

__device__ __forceinline__ bool interface_point(int nx, int ny, const double *r1, const double *r2,
                                                const uint8_t *solid, const int *par, const int *best2,
                                                const WallDesc &wd, long long a, int dir, double &qx_,
                                                double &qy_)
{
    const int x = (int)(a % nx), y = (int)(a / nx);
    const int x2 = x + (dir == 0), y2 = y + (dir == 1);
    if (x2 >= nx || y2 >= ny) return false;
    const long long b = (long long)y2 * nx + x2;
    if (solid[a] || solid[b]) return false;
    const double ra = (r1[a] - r2[a]) / (r1[a] + r2[a]);
    const double rb = (r1[b] - r2[b]) / (r1[b] + r2[b]);
    if ((ra > 0.0) == (rb > 0.0)) return false;
    if (par[a] != best2[ra > 0.0] || par[b] != best2[rb > 0.0]) return false;
    const double t = ra / (ra - rb);
    qx_ = x + t * (x2 - x);
    qy_ = y + t * (y2 - y);
    double dist;
    if (wd.kind == 0) {
        dist = qy_ - wd.w0;
    } else {
        const double dx = qx_ - wd.w0, dy = qy_ - wd.w1;
        dist = __builtin_sqrt(dx * dx + dy * dy) - wd.w2;
    }
    return dist >= 3.0;
}

template <int NV>
__device__ void block_sum(double (&v)[NV], double (*sh)[256])
{
    const int t = threadIdx.x;
    __syncthreads();
    for (int q = 0; q < NV; ++q) sh[q][t] = v[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int q = 0; q < NV; ++q) sh[q][t] += sh[q][t + h];
        __syncthreads();
    }
    for (int q = 0; q < NV; ++q) v[q] = sh[q][0];
}

static __device__ bool solve3(double A[3][3], double b[3], double x[3])
{
    double M[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) M[r][q] = A[r][q];
        M[r][3] = b[r];
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (__builtin_fabs(M[r][col]) > __builtin_fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return false;
        if (piv != col)
            for (int q = 0; q < 4; ++q) {
                const double tmp = M[col][q];
                M[col][q] = M[piv][q];
                M[piv][q] = tmp;
            }
        for (int r = col + 1; r < 3; ++r) {
            const double fct = M[r][col] / M[col][col];
            for (int q = col; q < 4; ++q) M[r][q] -= fct * M[col][q];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double s = M[r][3];
        for (int q = r + 1; q < 3; ++q) s -= M[r][q] * x[q];
        x[r] = s / M[r][r];
    }
    return true;
}

// One workgroup per run.  out[run*6]: theta (deg), centre x, centre y,
// radius, number of points, status (0 ok, 1 too few points, 2 fit failed).
static __global__ void __launch_bounds__(256)
k_contact_angle(const int *__restrict__ dims /* nx, ny per run */, const long long *__restrict__ offs,
                const double *__restrict__ rho1, const double *__restrict__ rho2,
                const uint8_t *__restrict__ solid, const int *__restrict__ par_all,
                const int *__restrict__ best, const WallDesc *__restrict__ walls, double *out)
{
    __shared__ double sh[9][256];
    __shared__ double params[4];
    __shared__ int flag;
    const int run = blockIdx.x, t = threadIdx.x;
    const int nx = dims[2 * run], ny = dims[2 * run + 1];
    const long long off = offs[run];
    const double *r1 = rho1 + off, *r2 = rho2 + off;
    const uint8_t *sd = solid + off;
    const int *par = par_all + off, *best2 = best + 2 * run;
    const WallDesc wd = walls[run];
    const long long N = (long long)nx * ny;

    // pass 1: count and mean
    double m[3] = {0, 0, 0};
    for (long long a = t; a < N; a += 256)
        for (int dir = 0; dir < 2; ++dir) {
            double qx_, qy_;
            if (interface_point(nx, ny, r1, r2, sd, par, best2, wd, a, dir, qx_, qy_)) {
                m[0] += 1.0;
                m[1] += qx_;
                m[2] += qy_;
            }
        }
    block_sum<3>(m, sh);
    double *o = out + (long long)run * 6;
    if (m[0] < 3.0) {
        if (t == 0) {
            o[0] = 0; o[1] = 0; o[2] = 0; o[3] = 0; o[4] = m[0]; o[5] = 1;
        }
        return;
    }
    const double mx = m[1] / m[0], my = m[2] / m[0];
    // pass 2: algebraic fit on centred points
    double k9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (long long a = t; a < N; a += 256)
        for (int dir = 0; dir < 2; ++dir) {
            double qx_, qy_;
            if (interface_point(nx, ny, r1, r2, sd, par, best2, wd, a, dir, qx_, qy_)) {
                const double u = qx_ - mx, v = qy_ - my, z = u * u + v * v;
                k9[0] += u * u; k9[1] += u * v; k9[2] += u;
                k9[3] += v * v; k9[4] += v;
                k9[5] += 1.0;
                k9[6] -= u * z; k9[7] -= v * z; k9[8] -= z;
            }
        }
    block_sum<9>(k9, sh);
    if (t == 0) {
        double A[3][3] = {{k9[0], k9[1], k9[2]}, {k9[1], k9[3], k9[4]}, {k9[2], k9[4], k9[5]}};
        double bb[3] = {k9[6], k9[7], k9[8]}, DEF[3];
        flag = 0;
        if (!solve3(A, bb, DEF)) flag = 2;
        const double r2v = DEF[0] * DEF[0] / 4.0 + DEF[1] * DEF[1] / 4.0 - DEF[2];
        if (!(r2v > 0.0)) flag = 2;
        params[0] = mx - DEF[0] / 2.0;
        params[1] = my - DEF[1] / 2.0;
        params[2] = flag ? 0.0 : __builtin_sqrt(r2v);
    }
    __syncthreads();
    if (flag) {
        if (t == 0) {
            o[0] = 0; o[1] = 0; o[2] = 0; o[3] = 0; o[4] = m[0]; o[5] = 2;
        }
        return;
    }
    // Gauss-Newton on the geometric distance
    for (int it = 0; it < 100; ++it) {
        const double a0 = params[0], b0 = params[1], rr = params[2];
        double g9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (long long a = t; a < N; a += 256)
            for (int dir = 0; dir < 2; ++dir) {
                double qx_, qy_;
                if (interface_point(nx, ny, r1, r2, sd, par, best2, wd, a, dir, qx_, qy_)) {
                    const double dx = qx_ - a0, dy = qy_ - b0;
                    const double d = __builtin_sqrt(dx * dx + dy * dy);
                    if (d == 0.0) continue;
                    const double J0 = -dx / d, J1 = -dy / d, J2 = -1.0, res = d - rr;
                    g9[0] += J0 * J0; g9[1] += J0 * J1; g9[2] += J0 * J2;
                    g9[3] += J1 * J1; g9[4] += J1 * J2; g9[5] += J2 * J2;
                    g9[6] -= J0 * res; g9[7] -= J1 * res; g9[8] -= J2 * res;
                }
            }
        block_sum<9>(g9, sh);
        if (t == 0) {
            double A[3][3] = {{g9[0], g9[1], g9[2]}, {g9[1], g9[3], g9[4]}, {g9[2], g9[4], g9[5]}};
            double bb[3] = {g9[6], g9[7], g9[8]}, dl[3];
            flag = 1;  // stop
            if (solve3(A, bb, dl)) {
                params[0] += dl[0];
                params[1] += dl[1];
                params[2] += dl[2];
                const double step = __builtin_fabs(dl[0]) + __builtin_fabs(dl[1]) + __builtin_fabs(dl[2]);
                flag = step <= 1e-13 * (1.0 + __builtin_fabs(params[2])) ? 1 : 0;
            }
        }
        __syncthreads();
        if (flag) break;
    }
    if (t == 0) {
        double cth;
        if (wd.kind == 0) {
            cth = -(params[1] - wd.w0) / params[2];
        } else {
            const double dx = params[0] - wd.w0, dy = params[1] - wd.w1;
            cth = (wd.w2 * wd.w2 + params[2] * params[2] - (dx * dx + dy * dy)) / (2.0 * wd.w2 * params[2]);
        }
        cth = cth > 1.0 ? 1.0 : (cth < -1.0 ? -1.0 : cth);
        o[0] = acos(cth) * (180.0 / 3.14159265358979323846);
        o[1] = params[0];
        o[2] = params[1];
        o[3] = params[2];
        o[4] = m[0];
        o[5] = 0;
    }
}

}  // namespace lbm
