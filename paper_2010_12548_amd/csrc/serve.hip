// serve.hip -- point-table preparation for serving: a row-major bucket grid,
// so that the points of a viewport are a few contiguous ranges.
#include "sba_internal.h"

__device__ __forceinline__ int32_t bucket_of(int32_t x, int32_t y, int64_t x0, int64_t y0,
                                             int64_t cell, int32_t G)
{
    int64_t bx = ((int64_t)x - x0), by = ((int64_t)y - y0);
    bx = bx < 0 ? 0 : bx / cell;
    by = by < 0 ? 0 : by / cell;
    if (bx >= G) bx = G - 1;
    if (by >= G) by = G - 1;
    return (int32_t)(by * G + bx);
}

__global__ void k_bucket_count(const int32_t *xy, int64_t n, int64_t x0, int64_t y0, int64_t cell,
                               int32_t G, int64_t *cnt)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd((unsigned long long *)&cnt[bucket_of(xy[2 * t], xy[2 * t + 1], x0, y0, cell, G)],
                  1ull);
}

__global__ void k_bucket_scatter(const int32_t *xy, const int64_t *vals, int64_t n, int64_t x0,
                                 int64_t y0, int64_t cell, int32_t G, int64_t *cursor,
                                 int32_t *oxy, int64_t *ovals)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = xy[2 * t], y = xy[2 * t + 1];
        int64_t pos = (int64_t)atomicAdd((unsigned long long *)&cursor[bucket_of(x, y, x0, y0, cell, G)],
                                         1ull);
        oxy[2 * pos] = x;
        oxy[2 * pos + 1] = y;
        if (vals) ovals[pos] = vals[t];
    }
}

__global__ void k_fill_i64(int64_t *a, int64_t n, int64_t v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

int bucket_launch(const int32_t *xy, const int64_t *values, int64_t n, int32_t x0, int32_t y0,
                  int32_t cell, int32_t G, int32_t *out_xy, int64_t *out_values, int64_t *off,
                  hipStream_t st)
{
    const int64_t nb = (int64_t)G * G;
    int64_t *cursor = nullptr;
    RC(tmp_alloc(&cursor, nb + 1, st));
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(nb + 1)), dim3(256), 0, st, off, nb + 1, (int64_t)0);
    unsigned g = (unsigned)std::min<int64_t>(grid_for(n), 4096);
    if (n > 0)
        hipLaunchKernelGGL(k_bucket_count, dim3(g), dim3(256), 0, st, xy, n, (int64_t)x0, (int64_t)y0,
                           (int64_t)cell, G, off);
    int rc = hipGetLastError() == hipSuccess ? 0 : SBA_EDEVICE;
    if (!rc) rc = scan_exclusive_i64(off, off, nb, off + nb, st);
    if (!rc && hipMemcpyAsync(cursor, off, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToDevice, st) !=
                   hipSuccess)
        rc = SBA_EDEVICE;
    if (!rc && n > 0) {
        hipLaunchKernelGGL(k_bucket_scatter, dim3(g), dim3(256), 0, st, xy, values, n, (int64_t)x0,
                           (int64_t)y0, (int64_t)cell, G, cursor, out_xy, out_values);
        if (hipGetLastError() != hipSuccess) rc = SBA_EDEVICE;
    }
    tmp_free(cursor, st);
    return rc;
}
