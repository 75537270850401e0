// Spatial order of the queries: which 64 queries share a tile.
//
// Every query is computed alone (Eq. 1-6 involve only the query and the data
// points), so any grouping of queries into waves gives each query its own
// result; the grouping decides the speed.  Pass 1 screens each 16-point batch
// against the list of every lane of the wave, so a batch costs an insertion
// round whenever one lane's list takes a point: with 64 neighbouring queries
// those rounds coincide.  Pass 2 takes the one-transcendental loop only where
// all 64 lanes share a whole power: on clustered data alpha follows the local
// density, so neighbouring queries mostly share it.
//
// The order: Morton codes of the queries' cells in a 2^b x 2^b grid over the
// bounding box of the problem's queries, sorted by a stable LSD radix sort
// with 8-bit digits (ties keep the caller's order).  Each pass is a digit
// histogram per sort block, an exclusive scan per problem (digit-major,
// then block), and a stable scatter in which each wave ranks its lanes among
// equal digits with ballots.  Counts and ranks do not depend on timing, so
// the order is the same on every run.  Several problems sort at once, each
// within its own range of positions (the scan runs over each problem's own
// histogram region).  No memset: every buffer is written before it is read,
// so the launches can be captured in a graph.
#include "common.h"

namespace aidw {

int order_bits(int64_t n) {
    if (n <= kWaveSize) return 0;
    // about 16 queries per cell on average (a tile then spans a few cells)
    int b = 1;
    while (b < 11 && (int64_t(1) << (2 * b)) * 16 < n) ++b;
    return b;
}

size_t order_workspace_bytes(int64_t total, int blocks, int segments, int passes, OrderLaunch* L,
                             char* base) {
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) / a * a; };
    const size_t e = (size_t)total;
    const int mid = passes > 2 ? 2 : (passes > 1 ? 1 : 0);  // intermediate key/value buffers
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += up(bytes);
        return base ? base + o : nullptr;
    };
    char* bbox = take(sizeof(float4) * (size_t)segments);
    char* part = take(sizeof(float4) * (size_t)blocks);
    char* hist = take(sizeof(int) * 256 * (size_t)blocks);
    char* order = take(sizeof(int) * e);
    char* keys[2] = {nullptr, nullptr};
    char* vals[2] = {nullptr, nullptr};
    for (int i = 0; i < mid; ++i) {
        keys[i] = take(sizeof(unsigned) * e);
        vals[i] = take(sizeof(int) * e);
    }
    if (L && base) {
        L->bbox = reinterpret_cast<float4*>(bbox);
        L->part = reinterpret_cast<float4*>(part);
        L->hist = reinterpret_cast<int*>(hist);
        L->order = reinterpret_cast<int*>(order);
        for (int i = 0; i < 2; ++i) {
            L->keys[i] = reinterpret_cast<unsigned*>(keys[i]);
            L->vals[i] = reinterpret_cast<int*>(vals[i]);
        }
    }
    return off;
}

namespace {

__device__ __forceinline__ OrderSeg segment(const OrderLaunch& L, int s) {
    return L.table ? L.table[s] : L.one;
}

__device__ __forceinline__ int block_segment(const OrderLaunch& L, int b) {
    return L.table ? L.block_seg[b] : 0;
}

// The low 16 bits of v spread to the even bit positions.
__device__ __forceinline__ unsigned spread_bits(unsigned v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Cell index along one axis: (v - lo) * scale clamped to [0, cells - 1]
// (NaN and infinite coordinates land in an edge cell; the order only
// groups queries, any cell is correct).
__device__ __forceinline__ unsigned cell_of(float v, float lo, float scale, float top) {
    const float t = fminf(fmaxf((v - lo) * scale, 0.0f), top);
    return (unsigned)t;
}

__device__ __forceinline__ unsigned morton_key(const OrderSeg& s, float4 bb, int i) {
    const float top = (float)((1 << s.bits) - 1);
    return spread_bits(cell_of(s.qx[i], bb.x, bb.z, top)) |
           (spread_bits(cell_of(s.qy[i], bb.y, bb.w, top)) << 1);
}

// Min and max of x and y over a wave (NaN ignored: fminf/fmaxf keep the
// other operand).
__device__ __forceinline__ void wave_box(float& x0, float& x1, float& y0, float& y1) {
    for (int o = kWaveSize / 2; o > 0; o >>= 1) {
        x0 = fminf(x0, __shfl_xor(x0, o));
        x1 = fmaxf(x1, __shfl_xor(x1, o));
        y0 = fminf(y0, __shfl_xor(y0, o));
        y1 = fmaxf(y1, __shfl_xor(y1, o));
    }
}

// Bounding box of the queries of one sort block, as (x0, x1, y0, y1).
__global__ __launch_bounds__(kOrderThreads) void aidw_order_box_part(OrderLaunch L) {
    constexpr int W = kOrderThreads / kWaveSize;
    __shared__ float red[4][W];
    const OrderSeg s = segment(L, block_segment(L, blockIdx.x));
    const int i0 = (blockIdx.x - s.block0) * kOrderBlock;
    const int i1 = min(s.n, i0 + kOrderBlock);
    float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kOrderThreads) {
        const float x = s.qx[i], y = s.qy[i];
        x0 = fminf(x0, x);
        x1 = fmaxf(x1, x);
        y0 = fminf(y0, y);
        y1 = fmaxf(y1, y);
    }
    wave_box(x0, x1, y0, y1);
    const int w = threadIdx.x / kWaveSize;
    if (threadIdx.x % kWaveSize == 0) {
        red[0][w] = x0;
        red[1][w] = x1;
        red[2][w] = y0;
        red[3][w] = y1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < W; ++v) {
            x0 = fminf(x0, red[0][v]);
            x1 = fmaxf(x1, red[1][v]);
            y0 = fminf(y0, red[2][v]);
            y1 = fmaxf(y1, red[3][v]);
        }
        L.part[blockIdx.x] = make_float4(x0, x1, y0, y1);
    }
}

// Each problem's box from its blocks' boxes, as (x0, y0, cells / width,
// cells / height); one wave per problem.
__global__ __launch_bounds__(kWaveSize) void aidw_order_bbox(OrderLaunch L) {
    const OrderSeg s = segment(L, blockIdx.x);
    float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int b = threadIdx.x; b < s.nblocks; b += kWaveSize) {
        const float4 v = L.part[s.block0 + b];
        x0 = fminf(x0, v.x);
        x1 = fmaxf(x1, v.y);
        y0 = fminf(y0, v.z);
        y1 = fmaxf(y1, v.w);
    }
    wave_box(x0, x1, y0, y1);
    if (threadIdx.x == 0) {
        const float cells = (float)(1 << s.bits);
        // zero scale for an empty, single-valued or non-finite extent
        const float sx = x1 > x0 ? __fdiv_rn(cells, x1 - x0) : 0.0f;
        const float sy = y1 > y0 ? __fdiv_rn(cells, y1 - y0) : 0.0f;
        L.bbox[blockIdx.x] =
            make_float4(x0, y0, sx < INFINITY ? sx : 0.0f, sy < INFINITY ? sy : 0.0f);
    }
}

// Where a pass finds the key of element i of segment s.
enum KeySource {
    kFromCoords = 0,  // first pass: the Morton code of the query's cell
    kFromPrev = 1,    // later passes: the previous pass's output
    kGiven = 2,       // a one-pass sort of keys the caller computed (value: i)
};

template <int SRC>
__device__ __forceinline__ void key_of(const OrderLaunch& L, const OrderSeg& s, int si, int i,
                                       const unsigned* keys_in, const int* vals_in, unsigned& key,
                                       int& val) {
    if constexpr (SRC == kFromCoords) {
        key = morton_key(s, L.bbox[si], i);
        val = i;
    } else if constexpr (SRC == kGiven) {
        key = keys_in[(int64_t)s.base + i];
        val = i;
    } else {
        key = keys_in[(int64_t)s.base + i];
        val = vals_in[(int64_t)s.base + i];
    }
}

// Digit counts of one sort block b: hist[256 * b + digit].
template <int SRC>
__global__ __launch_bounds__(kOrderThreads) void aidw_order_hist(OrderLaunch L, int shift,
                                                                 const unsigned* keys_in,
                                                                 const int* vals_in) {
    __shared__ int h[256];
    const int si = block_segment(L, blockIdx.x);
    const OrderSeg s = segment(L, si);
    const int lb = blockIdx.x - s.block0;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int i0 = lb * kOrderBlock;
    for (int c = 0; c < kOrderItems; ++c) {
        const int i = i0 + c * kOrderThreads + threadIdx.x;
        if (i < s.n) {
            unsigned key;
            int val;
            key_of<SRC>(L, s, si, i, keys_in, vals_in, key, val);
            atomicAdd(&h[(key >> shift) & 255u], 1);
        }
    }
    __syncthreads();
    L.hist[256 * (int64_t)blockIdx.x + threadIdx.x] = h[threadIdx.x];
}

// Counts to scatter offsets, one workgroup per problem: the first position
// of digit d of block b is base + (queries with a smaller digit) + (queries
// with digit d in earlier blocks).
__global__ __launch_bounds__(256) void aidw_order_scan(OrderLaunch L) {
    __shared__ int tot[256];
    const OrderSeg s = segment(L, blockIdx.x);
    const int d = threadIdx.x;
    int* h = L.hist + 256 * (int64_t)s.block0 + d;  // the problem's blocks are consecutive
    int run = 0;
    for (int b = 0; b < s.nblocks; ++b) {
        const int v = h[256 * b];
        h[256 * b] = run;
        run += v;
    }
    tot[d] = run;
    __syncthreads();
    // inclusive scan of the 256 digit totals (Hillis-Steele)
    for (int o = 1; o < 256; o <<= 1) {
        const int v = d >= o ? tot[d - o] : 0;
        __syncthreads();
        tot[d] += v;
        __syncthreads();
    }
    const int first = s.base + tot[d] - run;
    for (int b = 0; b < s.nblocks; ++b) h[256 * b] += first;
}

// Stable scatter of one sort block.  The block's queries go in chunks of 256
// (position order: chunk, then wave, then lane); within a wave a lane's rank
// among equal digits is the number of lower lanes with its digit (ballots on
// each digit bit); waves of a chunk and earlier chunks add their counts.
template <int SRC>
__global__ __launch_bounds__(kOrderThreads) void aidw_order_scatter(OrderLaunch L, int shift,
                                                                    const unsigned* keys_in,
                                                                    const int* vals_in,
                                                                    unsigned* keys_out,
                                                                    int* vals_out) {
    constexpr int W = kOrderThreads / kWaveSize;
    __shared__ int offs[256], run[256], wcnt[W][256];
    const int si = block_segment(L, blockIdx.x);
    const OrderSeg s = segment(L, si);
    const int lb = blockIdx.x - s.block0;
    const int t = threadIdx.x, w = t / kWaveSize, lane = t % kWaveSize;
    offs[t] = L.hist[256 * (int64_t)blockIdx.x + t];
    run[t] = 0;
#pragma unroll
    for (int v = 0; v < W; ++v) wcnt[v][t] = 0;
    __syncthreads();
    const unsigned long long lower = (1ull << lane) - 1ull;
    const int i0 = lb * kOrderBlock;
    for (int c = 0; c < kOrderItems; ++c) {
        if (i0 + c * kOrderThreads >= s.n) break;  // the same for the whole workgroup
        const int i = i0 + c * kOrderThreads + t;
        const bool valid = i < s.n;
        unsigned key = 0;
        int val = 0;
        if (valid) key_of<SRC>(L, s, si, i, keys_in, vals_in, key, val);
        const unsigned d = (key >> shift) & 255u;
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const unsigned long long b = __ballot(set);
            same &= set ? b : ~b;
        }
        const int rank = __popcll(same & lower);
        if (valid && rank == 0) wcnt[w][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int pre = run[d];
            for (int v = 0; v < w; ++v) pre += wcnt[v][d];
            const int dest = offs[d] + pre + rank;
            if (keys_out) keys_out[dest] = key;
            vals_out[dest] = val;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            add += wcnt[v][t];
            wcnt[v][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_query_order(const OrderLaunch& L, hipStream_t stream) {
    if (L.blocks <= 0 || L.passes <= 0) return hipSuccess;
    hipLaunchKernelGGL(aidw_order_box_part, dim3((unsigned)L.blocks), dim3(kOrderThreads), 0,
                       stream, L);
    hipLaunchKernelGGL(aidw_order_bbox, dim3((unsigned)L.segments), dim3(kWaveSize), 0, stream, L);
    for (int pass = 0; pass < L.passes; ++pass) {
        const int shift = 8 * pass;
        const bool first = pass == 0, last = pass == L.passes - 1;
        const unsigned* kin = first ? nullptr : L.keys[(pass - 1) & 1];
        const int* vin = first ? nullptr : L.vals[(pass - 1) & 1];
        unsigned* kout = last ? nullptr : L.keys[pass & 1];
        int* vout = last ? L.order : L.vals[pass & 1];
        if (first)
            hipLaunchKernelGGL((aidw_order_hist<kFromCoords>), dim3((unsigned)L.blocks),
                               dim3(kOrderThreads), 0, stream, L, shift, kin, vin);
        else
            hipLaunchKernelGGL((aidw_order_hist<kFromPrev>), dim3((unsigned)L.blocks),
                               dim3(kOrderThreads), 0, stream, L, shift, kin, vin);
        hipLaunchKernelGGL(aidw_order_scan, dim3((unsigned)L.segments), dim3(256), 0, stream, L);
        if (first)
            hipLaunchKernelGGL((aidw_order_scatter<kFromCoords>), dim3((unsigned)L.blocks),
                               dim3(kOrderThreads), 0, stream, L, shift, kin, vin, kout, vout);
        else
            hipLaunchKernelGGL((aidw_order_scatter<kFromPrev>), dim3((unsigned)L.blocks),
                               dim3(kOrderThreads), 0, stream, L, shift, kin, vin, kout, vout);
    }
    return hipGetLastError();
}

hipError_t launch_key_order(const unsigned* keys, int n, int* hist, int* order,
                            hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    OrderLaunch L{};
    const int blocks = (n + kOrderBlock - 1) / kOrderBlock;
    L.one = OrderSeg{nullptr, nullptr, n, 0, 0, blocks, 0};
    L.segments = 1;
    L.blocks = blocks;
    L.passes = 1;
    L.hist = hist;
    L.order = order;
    hipLaunchKernelGGL((aidw_order_hist<kGiven>), dim3((unsigned)blocks), dim3(kOrderThreads), 0,
                       stream, L, 0, keys, (const int*)nullptr);
    hipLaunchKernelGGL(aidw_order_scan, dim3(1), dim3(256), 0, stream, L);
    hipLaunchKernelGGL((aidw_order_scatter<kGiven>), dim3((unsigned)blocks), dim3(kOrderThreads), 0,
                       stream, L, 0, keys, (const int*)nullptr, (unsigned*)nullptr, order);
    return hipGetLastError();
}

}  // namespace aidw
