// k nearest neighbours through a uniform grid: an exact alternative to the
// full pass-1 scan (the region partitioning that the paper discusses and sets
// aside because its kNN runs inside one thread, Sec. 3.1.2).  Pass 2 is not
// affected: it still sums over all m points.
//
// Build (all on the device, no host round trip):
//   1. bounding box of the data (per-block partial min/max, then one block);
//   2. a grid of near-square cells over the box, about two points per cell;
//   3. counting sort of the points by cell (count, exclusive scan, scatter).
// Query (one query per lane): visit the cells in square rings around the
// query's cell; after ring r every unvisited point is at least (r - 1) cell
// widths away (one cell of slack covers rounding in the cell assignment), so
// the search stops once the k-th smallest squared distance is below that
// bound, reduced by a relative 2^-20 for the rounding of computed squared
// distances.  Squared distances use the same formula as the full scan, so the
// k-nearest multiset -- and with it r_obs, alpha and the pass-2 exponent
// terms -- are bit-identical to the full scan's.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "common.h"
#include "device_math.h"

namespace aidw {
namespace {

constexpr int kBlock = 256;

__global__ void bbox_partial(const float* __restrict__ x, const float* __restrict__ y, int m,
                             float4* __restrict__ part) {
    __shared__ float4 s[kBlock];
    float4 v = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        v.x = fminf(v.x, x[i]);
        v.y = fminf(v.y, y[i]);
        v.z = fmaxf(v.z, x[i]);
        v.w = fmaxf(v.w, y[i]);
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const float4 o = s[threadIdx.x + w];
            float4& a = s[threadIdx.x];
            a.x = fminf(a.x, o.x);
            a.y = fminf(a.y, o.y);
            a.z = fmaxf(a.z, o.z);
            a.w = fmaxf(a.w, o.w);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// One block: final bounding box and the grid geometry.  The cells are close
// to square and there are at most `cap` of them; an axis on which the data
// have no extent (or one too small for a normal cell size) gets one cell.
__global__ void grid_setup(const float4* __restrict__ part, int nparts, int cap, GridGeom* geo) {
    __shared__ float4 s[kBlock];
    float4 v = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        const float4 o = part[i];
        v.x = fminf(v.x, o.x);
        v.y = fminf(v.y, o.y);
        v.z = fmaxf(v.z, o.z);
        v.w = fmaxf(v.w, o.w);
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const float4 o = s[threadIdx.x + w];
            float4& a = s[threadIdx.x];
            a.x = fminf(a.x, o.x);
            a.y = fminf(a.y, o.y);
            a.z = fmaxf(a.z, o.z);
            a.w = fmaxf(a.w, o.w);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float4 b = s[0];
        const float wx = b.z - b.x, wy = b.w - b.y;
        const float kNormal = 1.17549435e-38f;
        bool ex = wx / (float)cap >= kNormal, ey = wy / (float)cap >= kNormal;
        int gx = 1, gy = 1;
        if (ex && ey) {
            const float f = sqrtf((float)cap * (wx / wy));
            gx = f >= (float)cap ? cap : (f < 1.0f ? 1 : (int)f);
            gy = max(1, cap / gx);
        } else if (ex) {
            gx = cap;
        } else if (ey) {
            gy = cap;
        }
        GridGeom g;
        g.gx = gx;
        g.gy = gy;
        g.x0 = b.x;
        g.y0 = b.y;
        g.cw = ex ? wx / (float)gx : 1.0f;
        g.ch = ey ? wy / (float)gy : 1.0f;
        g.inv_cw = 1.0f / g.cw;
        g.inv_ch = 1.0f / g.ch;
        *geo = g;
    }
}

__device__ __forceinline__ int cell_of(int cells, float v, float v0, float inv) {
    const float f = floorf((v - v0) * inv);
    // compare in float first: huge or NaN values go to the border cells
    if (!(f >= 0.0f)) return 0;
    if (f >= (float)(cells - 1)) return cells - 1;
    return (int)f;
}

__device__ __forceinline__ int cell_index(const GridGeom& g, float x, float y) {
    return cell_of(g.gy, y, g.y0, g.inv_ch) * g.gx + cell_of(g.gx, x, g.x0, g.inv_cw);
}

// Zero the cell counters with a kernel rather than hipMemsetAsync, so that
// the sequence stays correct if a caller captures it in a hipGraph.
__global__ void grid_clear(int* __restrict__ counts, int* __restrict__ cursor, int cells) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i <= cells; i += gridDim.x * kBlock) {
        counts[i] = 0;
        if (i < cells) cursor[i] = 0;
    }
}

__global__ void grid_count(const float* __restrict__ x, const float* __restrict__ y, int m,
                           const GridGeom* __restrict__ geo, int* __restrict__ counts) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const GridGeom g = *geo;
    const int c = cell_index(g, x[i], y[i]);
    atomicAdd(&counts[c], 1);
}

__global__ void grid_scatter(const float* __restrict__ x, const float* __restrict__ y, int m,
                             const GridGeom* __restrict__ geo, const int* __restrict__ start,
                             int* __restrict__ cursor, float2* __restrict__ sorted) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const GridGeom g = *geo;
    const int c = cell_index(g, x[i], y[i]);
    const int pos = start[c] + atomicAdd(&cursor[c], 1);
    sorted[pos] = make_float2(x[i], y[i]);
}

template <int K>
__device__ __forceinline__ void visit_cell(const float2* __restrict__ sorted,
                                           const int* __restrict__ start, int c, float qx,
                                           float qy, float (&top)[K]) {
    const int b = start[c], e = start[c + 1];
    for (int j = b; j < e; ++j) {
        const float2 p = sorted[j];
        const float d2 = sqdist(qx, qy, p.x, p.y);
        if (d2 < top[K - 1]) list_insert<K>(top, d2);
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void grid_knn(ProblemF32 p, const GridGeom* __restrict__ geo,
                                                   const int* __restrict__ start,
                                                   const float2* __restrict__ sorted,
                                                   float* __restrict__ qpar) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= p.n) return;
    const GridGeom g = *geo;
    const float qx = p.qx[q], qy = p.qy[q];
    const int ci = cell_of(g.gx, qx, g.x0, g.inv_cw), cj = cell_of(g.gy, qy, g.y0, g.inv_ch);
    const int pad = K - p.ap.k;
    float top[K];
#pragma unroll
    for (int i = 0; i < K; ++i) top[i] = i < pad ? -INFINITY : INFINITY;
    for (int r = 0;; ++r) {
        const int i0 = ci - r, i1 = ci + r, j0 = cj - r, j1 = cj + r;
        const int ia = max(i0, 0), ib = min(i1, g.gx - 1);
        for (int j = max(j0, 0); j <= min(j1, g.gy - 1); ++j) {
            if (j == j0 || j == j1) {  // top and bottom rows of the ring: every column
                for (int i = ia; i <= ib; ++i) visit_cell<K>(sorted, start, j * g.gx + i, qx, qy, top);
            } else {  // side columns only
                if (i0 >= 0) visit_cell<K>(sorted, start, j * g.gx + i0, qx, qy, top);
                if (i1 < g.gx && i1 != i0) visit_cell<K>(sorted, start, j * g.gx + i1, qx, qy, top);
            }
        }
        const bool all_x = i0 <= 0 && i1 >= g.gx - 1, all_y = j0 <= 0 && j1 >= g.gy - 1;
        if (all_x && all_y) break;  // every cell seen
        // an unvisited point lies outside the visited block in x or in y
        const float bx = all_x ? INFINITY : (float)(r - 1) * g.cw;
        const float by = all_y ? INFINITY : (float)(r - 1) * g.ch;
        const float bound = fminf(bx, by);
        if (r >= 1 && top[K - 1] <= bound * bound * (1.0f - 0x1p-20f)) break;
    }
    double r_obs, al;
    float na, aL0, d2min;
    query_power<K>(top, p.ap, r_obs, al, na, aL0, d2min);
    qpar[q] = na;
    qpar[p.n + q] = aL0;
    qpar[2 * p.n + q] = sqrtf(d2min);
    qpar[3 * p.n + q] = (float)integer_power(al, d2min);
    if (p.r_obs) p.r_obs[q] = r_obs;
    if (p.alpha) p.alpha[q] = al;
}

template <int K>
hipError_t launch_grid_knn(const ProblemF32& p, const GridWorkspace& ws, hipStream_t s) {
    hipLaunchKernelGGL((grid_knn<K>), dim3((unsigned)((p.n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, p, ws.geo, ws.start, ws.sorted, ws.qpar);
    return hipGetLastError();
}

}  // namespace

int grid_cells(int64_t m) {
    const int64_t c = (m + 1) / 2;  // about two points per cell
    return (int)std::min<int64_t>(std::max<int64_t>(c, 1), 1 << 24);
}

size_t grid_temp_bytes(int cells) {
    size_t bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (int*)nullptr, (int*)nullptr,
                                           cells + 1);
    return bytes;
}

hipError_t launch_grid_knn_all(const ProblemF32& p, const GridWorkspace& ws, hipStream_t s) {
    const int cells = ws.cells;
    const int nparts = ws.nparts;
    const unsigned gc = (unsigned)std::min<int64_t>(1024, ((int64_t)cells + kBlock) / kBlock);
    hipLaunchKernelGGL(grid_clear, dim3(gc), dim3(kBlock), 0, s, ws.counts, ws.cursor, cells);
    hipLaunchKernelGGL(bbox_partial, dim3(nparts), dim3(kBlock), 0, s, p.dx, p.dy, p.m, ws.part);
    hipLaunchKernelGGL(grid_setup, dim3(1), dim3(kBlock), 0, s, ws.part, nparts, cells, ws.geo);
    const unsigned gm = (unsigned)((p.m + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(grid_count, dim3(gm), dim3(kBlock), 0, s, p.dx, p.dy, p.m, ws.geo,
                       ws.counts);
    size_t tb = ws.temp_bytes;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(ws.temp, tb, ws.counts, ws.start, cells + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grid_scatter, dim3(gm), dim3(kBlock), 0, s, p.dx, p.dy, p.m, ws.geo,
                       ws.start, ws.cursor, ws.sorted);
    switch (k_bucket(p.ap.k)) {
        case 4: return launch_grid_knn<4>(p, ws, s);
        case 8: return launch_grid_knn<8>(p, ws, s);
        case 10: return launch_grid_knn<10>(p, ws, s);
        case 12: return launch_grid_knn<12>(p, ws, s);
        case 16: return launch_grid_knn<16>(p, ws, s);
        case 20: return launch_grid_knn<20>(p, ws, s);
        case 24: return launch_grid_knn<24>(p, ws, s);
        case 32: return launch_grid_knn<32>(p, ws, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace aidw
