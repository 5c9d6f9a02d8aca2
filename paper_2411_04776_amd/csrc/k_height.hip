// k_height.hip -- height map of the deformed gel surface, the input of the
// optical tactile renderers the paper pairs with the soft-body gel (its
// Taxim / FOTS pipeline works on a height map of the sensing surface).
//
// For every pixel centre (x0 + i dx, y0 + j dy) the map holds
// z_ref - (the largest z at which the vertical line through the centre meets
// an upward-facing gel surface triangle), 0 where it meets none: the
// indentation depth below the reference height. Upward-facing: positive
// signed xy area, the surface triangles being oriented outward. Triangles are
// rasterised one per thread over their xy bounding box (widened by one
// pixel); a pixel is inside when its three edge functions are >= 0, z is the
// barycentric interpolation. The maximum is taken with
// 64-bit atomics on an order-preserving integer image of the FP64 height, so
// the map does not depend on the order of the threads.
#include "device_util.h"
#include "ipc_internal.h"

namespace ipcg {

// order-preserving map of doubles to unsigned 64-bit keys (0 = no hit)
__device__ __forceinline__ unsigned long long z_key(double z)
{
    long long b = __double_as_longlong(z);
    return b >= 0 ? ((unsigned long long)b | 0x8000000000000000ull) : ~(unsigned long long)b;
}

__device__ __forceinline__ double key_z(unsigned long long k)
{
    long long b = (k & 0x8000000000000000ull) ? (long long)(k & 0x7fffffffffffffffull) : (long long)~k;
    return __longlong_as_double(b);
}

__global__ void k_height_clear(unsigned long long *key, int64_t np)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) key[p] = 0ull;
}

__global__ void k_height_raster(const double *__restrict__ x, const int32_t *__restrict__ trv, int n_tris,
                                int n_gel_tris, HeightSpec hs, unsigned long long *key)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_gel_tris) return;
    const double *a = x + 3 * (int64_t)trv[t], *b = x + 3 * (int64_t)trv[n_tris + t],
                 *c = x + 3 * (int64_t)trv[2 * (int64_t)n_tris + t];
    double area = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
    if (!(area > 0.0)) return;  // facing down, vertical or degenerate
    double lox = fmin(a[0], fmin(b[0], c[0])), hix = fmax(a[0], fmax(b[0], c[0]));
    double loy = fmin(a[1], fmin(b[1], c[1])), hiy = fmax(a[1], fmax(b[1], c[1]));
    double fi0 = floor((lox - hs.x0) / hs.dx) - 1.0, fi1 = ceil((hix - hs.x0) / hs.dx) + 1.0;
    double fj0 = floor((loy - hs.y0) / hs.dy) - 1.0, fj1 = ceil((hiy - hs.y0) / hs.dy) + 1.0;
    if (!(fi1 >= 0.0) || !(fj1 >= 0.0) || !(fi0 < (double)hs.nx) || !(fj0 < (double)hs.ny)) return;
    int i0 = (int)fmax(fi0, 0.0), i1 = (int)fmin(fi1, (double)(hs.nx - 1));
    int j0 = (int)fmax(fj0, 0.0), j1 = (int)fmin(fj1, (double)(hs.ny - 1));
    for (int j = j0; j <= j1; ++j) {
        double py = hs.y0 + j * hs.dy;
        for (int i = i0; i <= i1; ++i) {
            double px = hs.x0 + i * hs.dx;
            double w0 = (c[0] - b[0]) * (py - b[1]) - (c[1] - b[1]) * (px - b[0]);
            double w1 = (a[0] - c[0]) * (py - c[1]) - (a[1] - c[1]) * (px - c[0]);
            double w2 = (b[0] - a[0]) * (py - a[1]) - (b[1] - a[1]) * (px - a[0]);
            if (!(w0 >= 0.0 && w1 >= 0.0 && w2 >= 0.0)) continue;
            double z = (w0 * a[2] + w1 * b[2] + w2 * c[2]) / area;
            atomicMax(&key[(int64_t)j * hs.nx + i], z_key(z));
        }
    }
}

__global__ void k_height_out(const unsigned long long *key, int64_t np, double z_ref, double *out)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    unsigned long long k = key[p];
    out[p] = k ? z_ref - key_z(k) : 0.0;
}

void launch_height_map(Scene &s, const HeightSpec &hs, unsigned long long *key, double *out, hipStream_t strm)
{
    int64_t np = (int64_t)hs.nx * hs.ny;
    int nb = (int)((np + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_height_clear, dim3(nb), dim3(kBlock), 0, strm, key, np);
    if (s.n_gel_tris > 0)
        hipLaunchKernelGGL(k_height_raster, dim3(nblocks(s.n_gel_tris)), dim3(kBlock), 0, strm, s.h.x, s.h.trv,
                           s.h.n_tris, s.n_gel_tris, hs, key);
    hipLaunchKernelGGL(k_height_out, dim3(nb), dim3(kBlock), 0, strm, key, np, hs.z_ref, out);
}

}  // namespace ipcg
