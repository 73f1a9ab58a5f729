// Contact angle of a droplet on a 3-D lattice (FP64, on the device): phase
// regions, interface points of rho^e = 0 along x, y and z links, sphere fit
// (arXiv 2505.22256, Sec. 3.5; the paper does not state how it measures the
// angle).  Reads the rho1 / rho2 fields of the 3-D fields pass.
#pragma once

#include "lbm_contact.hpp"

namespace lbm3 {

struct Wall3 {
    int kind;  // 0: flat wall z = w[0]; 1: sphere of centre w[0..2], surface radius w[3]
    double w[4];
};

__device__ __forceinline__ bool positive3(const double *r1, const double *r2, long long a)
{
    return (r1[a] - r2[a]) / (r1[a] + r2[a]) > 0.0;
}

// Union-find over fluid nodes: 6-connected regions of one phase, links not
// across periodic seams; every root is its region's smallest node.
static __global__ void __launch_bounds__(256)
k_cc3_init(long long N, const uint8_t *__restrict__ solid, int *__restrict__ par, int *__restrict__ cnt)
{
    for (long long a = (long long)blockIdx.x * 256 + threadIdx.x; a < N; a += (long long)gridDim.x * 256) {
        par[a] = solid[a] ? -1 : (int)a;
        cnt[a] = 0;
    }
}

static __global__ void __launch_bounds__(256)
k_cc3_hook(int nx, int ny, int nz, const double *__restrict__ r1, const double *__restrict__ r2,
           const uint8_t *__restrict__ solid, int *par)
{
    const long long N = (long long)nx * ny * nz, plane = (long long)nx * ny;
    for (long long a = (long long)blockIdx.x * 256 + threadIdx.x; a < N; a += (long long)gridDim.x * 256) {
        if (solid[a]) continue;
        const int x = (int)(a % nx), y = (int)((a / nx) % ny), z = (int)(a / plane);
        const bool pa = positive3(r1, r2, a);
        if (x + 1 < nx && !solid[a + 1] && positive3(r1, r2, a + 1) == pa) lbm::cc_unite(par, (int)a, (int)(a + 1));
        if (y + 1 < ny && !solid[a + nx] && positive3(r1, r2, a + nx) == pa) lbm::cc_unite(par, (int)a, (int)(a + nx));
        if (z + 1 < nz && !solid[a + plane] && positive3(r1, r2, a + plane) == pa)
            lbm::cc_unite(par, (int)a, (int)(a + plane));
    }
}

static __global__ void __launch_bounds__(256)
k_cc3_count(long long N, const uint8_t *__restrict__ solid, int *par, int *cnt)
{
    for (long long a = (long long)blockIdx.x * 256 + threadIdx.x; a < N; a += (long long)gridDim.x * 256) {
        if (solid[a]) continue;
        int r = (int)a;
        while (par[r] != r) r = par[r];
        par[a] = r;
        atomicAdd(cnt + r, 1);
    }
}

// best[phase] = root of the largest region of that phase (ties: the
// smaller root), -1 when absent; one workgroup.
static __global__ void __launch_bounds__(256)
k_cc3_pick(long long N, const double *__restrict__ r1, const double *__restrict__ r2, const uint8_t *__restrict__ solid,
           const int *__restrict__ par, const int *__restrict__ cnt, int *__restrict__ best)
{
    __shared__ unsigned long long sh[2][256];
    const int t = threadIdx.x;
    unsigned long long key[2] = {0ull, 0ull};
    for (long long a = t; a < N; a += 256) {
        if (solid[a] || par[a] != (int)a) continue;
        const int ph = positive3(r1, r2, a) ? 1 : 0;
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
        best[t] = k ? (int)(0xffffffffull - (k & 0xffffffffull)) : -1;
    }
}

__device__ __forceinline__ bool point3(int nx, int ny, int nz, const double *r1, const double *r2, const uint8_t *solid,
                                       const int *par, const int *best, const Wall3 &wd, long long a, int dir,
                                       double &px, double &py, double &pz)
{
    const long long plane = (long long)nx * ny;
    const int x = (int)(a % nx), y = (int)((a / nx) % ny), z = (int)(a / plane);
    const int x2 = x + (dir == 0), y2 = y + (dir == 1), z2 = z + (dir == 2);
    if (x2 >= nx || y2 >= ny || z2 >= nz) return false;
    const long long b = ((long long)z2 * ny + y2) * nx + x2;
    if (solid[a] || solid[b]) return false;
    const double ra = (r1[a] - r2[a]) / (r1[a] + r2[a]);
    const double rb = (r1[b] - r2[b]) / (r1[b] + r2[b]);
    if ((ra > 0.0) == (rb > 0.0)) return false;
    if (par[a] != best[ra > 0.0] || par[b] != best[rb > 0.0]) return false;
    const double tp = ra / (ra - rb);
    px = x + tp * (x2 - x);
    py = y + tp * (y2 - y);
    pz = z + tp * (z2 - z);
    double dist;
    if (wd.kind == 0) {
        dist = pz - wd.w[0];
    } else {
        const double dx = px - wd.w[0], dy = py - wd.w[1], dz = pz - wd.w[2];
        dist = __builtin_sqrt(dx * dx + dy * dy + dz * dz) - wd.w[3];
    }
    return dist >= 3.0;
}

static __device__ bool solve4(double A[4][4], double b[4], double x[4])
{
    double M[4][5];
    for (int r = 0; r < 4; ++r) {
        for (int q = 0; q < 4; ++q) M[r][q] = A[r][q];
        M[r][4] = b[r];
    }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (__builtin_fabs(M[r][col]) > __builtin_fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return false;
        if (piv != col)
            for (int q = 0; q < 5; ++q) {
                const double tmp = M[col][q];
                M[col][q] = M[piv][q];
                M[piv][q] = tmp;
            }
        for (int r = col + 1; r < 4; ++r) {
            const double fct = M[r][col] / M[col][col];
            for (int q = col; q < 5; ++q) M[r][q] -= fct * M[col][q];
        }
    }
    for (int r = 3; r >= 0; --r) {
        double s = M[r][4];
        for (int q = r + 1; q < 4; ++q) s -= M[r][q] * x[q];
        x[r] = s / M[r][r];
    }
    return true;
}

// One workgroup of 256 threads: out = theta (deg), centre (3), radius,
// number of points, status (0 ok, 1 too few points, 2 fit failed).  Every
// pass recomputes the points in a fixed order per thread and sums with a
// fixed tree, so the result is deterministic.
static __global__ void __launch_bounds__(256)
k_contact3(int nx, int ny, int nz, const double *__restrict__ r1, const double *__restrict__ r2,
           const uint8_t *__restrict__ solid, const int *__restrict__ par, const int *__restrict__ best, Wall3 wd,
           double *out)
{
    __shared__ double sh[14][256];
    __shared__ double prm[4];
    __shared__ int flag;
    const int t = threadIdx.x;
    const long long N = (long long)nx * ny * nz;
    double m[4] = {0, 0, 0, 0};
    for (long long a = t; a < N; a += 256)
        for (int dir = 0; dir < 3; ++dir) {
            double px, py, pz;
            if (point3(nx, ny, nz, r1, r2, solid, par, best, wd, a, dir, px, py, pz)) {
                m[0] += 1.0;
                m[1] += px;
                m[2] += py;
                m[3] += pz;
            }
        }
    lbm::block_sum<4>(m, sh);
    if (m[0] < 4.0) {
        if (t == 0) {
            for (int q = 0; q < 5; ++q) out[q] = 0.0;
            out[5] = m[0];
            out[6] = 1;
        }
        return;
    }
    const double mx = m[1] / m[0], my = m[2] / m[0], mz = m[3] / m[0];
    // algebraic fit x^2 + y^2 + z^2 + D x + E y + F z + G = 0 on centred points
    double k14[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (long long a = t; a < N; a += 256)
        for (int dir = 0; dir < 3; ++dir) {
            double px, py, pz;
            if (point3(nx, ny, nz, r1, r2, solid, par, best, wd, a, dir, px, py, pz)) {
                const double u = px - mx, v = py - my, w = pz - mz, s = u * u + v * v + w * w;
                k14[0] += u * u; k14[1] += u * v; k14[2] += u * w; k14[3] += u;
                k14[4] += v * v; k14[5] += v * w; k14[6] += v;
                k14[7] += w * w; k14[8] += w;
                k14[9] += 1.0;
                k14[10] -= u * s; k14[11] -= v * s; k14[12] -= w * s; k14[13] -= s;
            }
        }
    lbm::block_sum<14>(k14, sh);
    if (t == 0) {
        double A[4][4] = {{k14[0], k14[1], k14[2], k14[3]}, {k14[1], k14[4], k14[5], k14[6]},
                          {k14[2], k14[5], k14[7], k14[8]}, {k14[3], k14[6], k14[8], k14[9]}};
        double bb[4] = {k14[10], k14[11], k14[12], k14[13]}, D[4] = {0, 0, 0, 0};
        flag = solve4(A, bb, D) ? 0 : 2;
        const double r2v = (D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) / 4.0 - D[3];
        if (!(r2v > 0.0)) flag = 2;
        prm[0] = mx - D[0] / 2.0;
        prm[1] = my - D[1] / 2.0;
        prm[2] = mz - D[2] / 2.0;
        prm[3] = flag ? 0.0 : __builtin_sqrt(r2v);
    }
    __syncthreads();
    if (flag) {
        if (t == 0) {
            for (int q = 0; q < 5; ++q) out[q] = 0.0;
            out[5] = m[0];
            out[6] = 2;
        }
        return;
    }
    // Gauss-Newton on the geometric distances
    for (int it = 0; it < 100; ++it) {
        const double cx = prm[0], cy = prm[1], cz = prm[2], rr = prm[3];
        double g14[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (long long a = t; a < N; a += 256)
            for (int dir = 0; dir < 3; ++dir) {
                double px, py, pz;
                if (point3(nx, ny, nz, r1, r2, solid, par, best, wd, a, dir, px, py, pz)) {
                    const double dx = px - cx, dy = py - cy, dz = pz - cz;
                    const double d = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
                    if (d == 0.0) continue;
                    const double J[4] = {-dx / d, -dy / d, -dz / d, -1.0};
                    const double res = d - rr;
                    g14[0] += J[0] * J[0]; g14[1] += J[0] * J[1]; g14[2] += J[0] * J[2]; g14[3] += J[0] * J[3];
                    g14[4] += J[1] * J[1]; g14[5] += J[1] * J[2]; g14[6] += J[1] * J[3];
                    g14[7] += J[2] * J[2]; g14[8] += J[2] * J[3];
                    g14[9] += J[3] * J[3];
                    g14[10] -= J[0] * res; g14[11] -= J[1] * res; g14[12] -= J[2] * res; g14[13] -= J[3] * res;
                }
            }
        lbm::block_sum<14>(g14, sh);
        if (t == 0) {
            double A[4][4] = {{g14[0], g14[1], g14[2], g14[3]}, {g14[1], g14[4], g14[5], g14[6]},
                              {g14[2], g14[5], g14[7], g14[8]}, {g14[3], g14[6], g14[8], g14[9]}};
            double bb[4] = {g14[10], g14[11], g14[12], g14[13]}, dl[4];
            flag = 1;
            if (solve4(A, bb, dl)) {
                for (int q = 0; q < 4; ++q) prm[q] += dl[q];
                const double step = __builtin_fabs(dl[0]) + __builtin_fabs(dl[1]) + __builtin_fabs(dl[2]) +
                                    __builtin_fabs(dl[3]);
                flag = step <= 1e-13 * (1.0 + __builtin_fabs(prm[3])) ? 1 : 0;
            }
        }
        __syncthreads();
        if (flag) break;
    }
    if (t == 0) {
        double cth;
        if (wd.kind == 0) {
            cth = -(prm[2] - wd.w[0]) / prm[3];
        } else {
            const double dx = prm[0] - wd.w[0], dy = prm[1] - wd.w[1], dz = prm[2] - wd.w[2];
            cth = (wd.w[3] * wd.w[3] + prm[3] * prm[3] - (dx * dx + dy * dy + dz * dz)) / (2.0 * wd.w[3] * prm[3]);
        }
        cth = cth > 1.0 ? 1.0 : (cth < -1.0 ? -1.0 : cth);
        out[0] = acos(cth) * (180.0 / 3.14159265358979323846);
        for (int q = 0; q < 4; ++q) out[1 + q] = prm[q];
        out[5] = m[0];
        out[6] = 0;
    }
}

}  // namespace lbm3
