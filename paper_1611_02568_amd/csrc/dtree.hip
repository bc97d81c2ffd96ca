// The data-driven quadtree of Barnes-Hut-SNE (the D-Quadtree, Section 3.3,
// Eq. 9-10) on gfx950, the tree PixelSNE replaces with the pixel-aligned one.
//
// The root spans the data, [min y_d, max y_d + eps) per axis; the screen
// scaling of Section 4.2 maps exactly that box onto [0, r)^2, so in the pixel
// frame the root is the screen.  Cells split into four equal quadrants until
// each leaf holds one point.  Positions are placed on a 2^32 x 2^32 grid over
// the root (q = floor(z 2^(32 - L)), exact for FP32 and FP64 positions) and
// keyed by 64-bit Morton codes; points that fall in one grid cell cannot be
// split there and share a leaf.  After the sort:
//
//   * a run of equal keys is one leaf; its level is the first level at which
//     the run's cell holds no other key: max of the levels at which its key
//     parts from the previous run and from the next one;
//   * the run's head starts a cell at every level from the one where its key
//     parts from the previous run down to its leaf level;
//   * cells are numbered per level in key order; the children of a cell are
//     the cells of the next level that start inside it, consecutive, so each
//     cell records the first cell of the next level at or after its start
//     (its first child if it has any) and its children are [cursor[g],
//     cursor[g + 1]).
//
// Counts and FP64 coordinate sums are reduced bottom-up as in the pixel tree
// (leaves in position order, inner cells over their children in child order),
// and the same traversal walks the result: it tells leaves by their missing
// children and takes a cell side of 2^(L - level) pixels at any depth.  The
// whole tree is rebuilt from scratch every iteration, as Barnes-Hut-SNE does.
#include "ctx.h"

namespace psne {

namespace {

constexpr int kBlock = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kBlock * kRsItems;
constexpr int kTopLevel = 5;
constexpr int kTopThreads = 1024;

inline dim3 grid_for(int64_t n) { return dim3((unsigned)ceil_div(n > 0 ? n : 1, kBlock)); }
inline bool fp64(const pixelsne_ctx* c) { return c->prm.precision == PSNE_FP64; }

__device__ __forceinline__ uint64_t spread_bits32(uint32_t v) {
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// grid coordinate of a position in [0, 2^L): floor(z 2^(32 - L)), exact
__device__ __forceinline__ uint32_t grid32(float z, int L) {
    return (uint32_t)ldexpf(z, 32 - L);
}
__device__ __forceinline__ uint32_t grid32(double z, int L) {
    return (uint32_t)ldexp(z, 32 - L);
}

// pending screen scaling, then the 64-bit grid key (x in even bits)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_snap64(const T* __restrict__ zh, T* __restrict__ z,
                                                   uint64_t* __restrict__ key,
                                                   uint32_t* __restrict__ idx,
                                                   const DevScalars* __restrict__ sc, int64_t n,
                                                   int r, int L) {
    using V = v2_t<T>;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const V p = norm_pos<T>(zh, sc, i, r);
    reinterpret_cast<V*>(z)[i] = p;
    key[i] = spread_bits32(grid32(p.x, L)) | (spread_bits32(grid32(p.y, L)) << 1);
    idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (64-bit key, index), 8-bit digits, 8 passes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_rs_hist64(const uint64_t* __restrict__ keys,
                                                      int64_t n, int shift,
                                                      uint32_t* __restrict__ hist,
                                                      int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int j = 0; j < kRsItems; j++) {
        const int64_t p = base + j * kBlock + threadIdx.x;
        if (p < n) atomicAdd(&h[(uint32_t)(keys[p] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one pass: digit bases from the scanned digit totals and the
// block's scanned histogram column; within a tile of 256, the rank of an item
// among the items of its digit comes from eight ballots (items in position
// order), so equal digits keep their order.
__global__ __launch_bounds__(kBlock) void k_rs_scatter64(const uint64_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin,
                                                         uint64_t* __restrict__ kout,
                                                         uint32_t* __restrict__ vout, int64_t n,
                                                         int shift,
                                                         const uint32_t* __restrict__ hist,
                                                         const uint32_t* __restrict__ dtot,
                                                         int64_t nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    {
        const uint32_t v = dtot[t];
        uint32_t x = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wcnt[0][w] = x;
        __syncthreads();
        uint32_t pre = x - v;
        for (int q = 0; q < w; q++) pre += wcnt[0][q];
        run[t] = pre + hist[(int64_t)t * nblocks + blockIdx.x];
        __syncthreads();
    }
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int j = 0; j < kRsItems; j++) {
        const int64_t p = base + j * kBlock + t;
        const bool valid = p < n;
        const uint64_t key = valid ? kin[p] : 0ull;
        const uint32_t val = valid ? (vin ? vin[p] : (uint32_t)p) : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
        __syncthreads();
        uint64_t peers = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = ballot64(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d] + rank;
            for (int q = 0; q < w; q++) off += wcnt[q][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    }
}

// ---------------------------------------------------------------------------
// cells
// ---------------------------------------------------------------------------
// first level at which sorted position s is in another cell than s - 1
// (0 for s = 0; kDLevels + 1 when the keys are equal)
__device__ __forceinline__ int first_new_level64(const uint64_t* __restrict__ keys, int64_t s) {
    if (s == 0) return 0;
    const uint64_t x = keys[s] ^ keys[s - 1];
    if (x == 0) return kDLevels + 1;
    const int hb = 63 - __clzll((long long)x);
    return kDLevels - (hb >> 1);
}

// For the head of a run of equal keys (a leaf): the level at which its cells
// start (l0) and its leaf level (ll); the run's last position in *tail.
// Returns false for positions inside a run.
__device__ __forceinline__ bool run_levels(const uint64_t* __restrict__ keys, int64_t n, int64_t s,
                                           int& l0, int& ll, int64_t* tail) {
    l0 = first_new_level64(keys, s);
    if (l0 > kDLevels) return false;
    int64_t t = s;
    const uint64_t k = keys[s];
    while (t + 1 < n && keys[t + 1] == k) t++;
    const int dn = t + 1 < n ? first_new_level64(keys, t + 1) : 0;
    ll = l0 > dn ? l0 : dn;
    if (ll > kDLevels) ll = kDLevels;
    *tail = t;
    return true;
}

// cells that start at each level, per block (rows: levels 0..32)
__global__ __launch_bounds__(kBlock) void k_dtree_count(const uint64_t* __restrict__ keys,
                                                        int64_t n, uint32_t* __restrict__ cnt,
                                                        int64_t nb) {
    __shared__ uint32_t wc[4][kMaxLevelsAll];
    const int t = threadIdx.x, w = t >> 6;
    const int64_t s = (int64_t)blockIdx.x * kBlock + t;
    int l0 = kDLevels + 1, ll = -1;
    int64_t tail = 0;
    if (!(s < n && run_levels(keys, n, s, l0, ll, &tail))) {
        l0 = kDLevels + 1;
        ll = -1;
    }
    for (int l = 0; l <= kDLevels; l++) {
        const uint64_t b = ballot64(l0 <= l && l <= ll);
        if (lane_id() == 0) wc[w][l] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (t <= kDLevels)
        cnt[(int64_t)t * nb + blockIdx.x] = wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
}

// Number the cells: a run head writes each cell it starts (start position,
// level, cursor = first cell of the next level at or after the start), and
// every position its leaf and its coordinates in sorted order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dtree_nodes(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ perm,
    const T* __restrict__ z, int64_t n, const uint32_t* __restrict__ off, int64_t nb,
    const uint32_t* __restrict__ ltot, DevScalars* __restrict__ sc, Node* __restrict__ nodes,
    uint32_t* __restrict__ cursor, uint32_t* __restrict__ leaf_of, T* __restrict__ zs) {
    using V = v2_t<T>;
    __shared__ uint32_t wc[4][kMaxLevelsAll];
    __shared__ uint32_t lbase[kMaxLevelsAll + 1];
    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    if (t == 0) {
        uint32_t b = 0;
        for (int l = 0; l <= kDLevels; l++) {
            lbase[l] = b;
            b += ltot[l];
        }
        lbase[kDLevels + 1] = b;
        if (blockIdx.x == 0) {
            for (int l = 0; l <= kDLevels; l++) {
                sc->level_size[l] = ltot[l];
                sc->level_base[l] = lbase[l];
            }
            sc->level_base[kDLevels + 1] = b;
            sc->n_nodes = b;
        }
    }
    const int64_t s = (int64_t)blockIdx.x * kBlock + t;
    int l0 = kDLevels + 1, ll = -1;
    int64_t tail = s;
    const bool head = s < n && run_levels(keys, n, s, l0, ll, &tail);
    if (!head) {
        l0 = kDLevels + 1;
        ll = -1;
    }
    for (int l = 0; l <= kDLevels; l++) {
        const uint64_t b = ballot64(l0 <= l && l <= ll);
        if (lane == 0) wc[w][l] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    const uint64_t le = lanemask_lt() | (1ull << lane);
    // inclusive count of cell starts up to s at each level
    uint32_t incl[kMaxLevelsAll];
#pragma unroll
    for (int l = 0; l <= kDLevels; l++) {
        const uint64_t b = ballot64(l0 <= l && l <= ll);
        uint32_t r = off[(int64_t)l * nb + blockIdx.x] + (uint32_t)__popcll(b & le);
        for (int q = 0; q < w; q++) r += wc[q][l];
        incl[l] = r;
    }
    if (s < n) reinterpret_cast<V*>(zs)[s] = reinterpret_cast<const V*>(z)[perm[s]];
    if (!head) return;
#pragma unroll
    for (int l = 0; l <= kDLevels; l++) {
        if (l0 <= l && l <= ll) {
            const uint32_t gid = lbase[l] + incl[l] - 1u;
            nodes[gid].start = (uint32_t)s;
            nodes[gid].level = (uint32_t)l;
            uint32_t cur = lbase[kDLevels + 1];
            if (l < kDLevels) {
                // starts of level l + 1 before s; s itself starts one there iff l + 1 <= ll
                const uint32_t before = incl[l + 1] - (l + 1 <= ll ? 1u : 0u);
                cur = lbase[l + 1] + before;
            }
            cursor[gid] = cur;
        }
    }
    const uint32_t leaf = lbase[ll] + incl[ll] - 1u;
    for (int64_t q = s; q <= tail; q++) leaf_of[q] = leaf;
}

__device__ __forceinline__ void put_cell(Node* __restrict__ nodes, CellF* __restrict__ c32,
                                         double2* __restrict__ nsum, uint32_t g, double sx,
                                         double sy, uint32_t count, uint32_t child, float rs0,
                                         float rs1) {
    const double cx = sx / (double)count, cy = sy / (double)count;
    nodes[g].cx = cx;
    nodes[g].cy = cy;
    nodes[g].count = count;
    nodes[g].child = child;
    nsum[g] = double2{sx, sy};
    if (c32) c32[g] = CellF{(float)cx * rs0, (float)cy * rs1, (float)count, child};
}

// Leaves: a run head sums its run's positions in order (FP64).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dtree_leaves(const uint64_t* __restrict__ keys,
                                                         const T* __restrict__ zs, int64_t n,
                                                         const uint32_t* __restrict__ leaf_of,
                                                         Node* __restrict__ nodes,
                                                         CellF* __restrict__ c32,
                                                         double2* __restrict__ nsum,
                                                         const DevScalars* __restrict__ sc) {
    using V = v2_t<T>;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n || first_new_level64(keys, s) > kDLevels) return;
    double sx = 0.0, sy = 0.0;
    int64_t q = s;
    const uint64_t k = keys[s];
    do {
        const V p = reinterpret_cast<const V*>(zs)[q];
        sx += (double)p.x;
        sy += (double)p.y;
        q++;
    } while (q < n && keys[q] == k);
    put_cell(nodes, c32, nsum, leaf_of[s], sx, sy, (uint32_t)(q - s), 0u, cell_scale(sc->s[0]),
             cell_scale(sc->s[1]));
}

// One cell of level l: its children are [cursor[g], cursor[g + 1]) (the end
// of the next level for the level's last cell); none means a leaf, written
// by k_dtree_leaves.  Counts and sums over the children in child order.
__device__ __forceinline__ void dtree_inner(int l, const DevScalars* __restrict__ sc,
                                            const uint32_t* __restrict__ cursor,
                                            Node* __restrict__ nodes, CellF* __restrict__ c32,
                                            double2* __restrict__ nsum, uint32_t t, uint32_t m,
                                            float rs0, float rs1) {
    const uint32_t g = sc->level_base[l] + t;
    const uint32_t fc = cursor[g];
    const uint32_t lc = (t + 1 < m) ? cursor[g + 1] : sc->level_base[l + 1] + sc->level_size[l + 1];
    if (lc <= fc) return;
    double ax = 0.0, ay = 0.0;
    uint32_t c = 0;
    for (uint32_t q = fc; q < lc; q++) {
        const double2 v = nsum[q];
        ax += v.x;
        ay += v.y;
        c += nodes[q].count;
    }
    put_cell(nodes, c32, nsum, g, ax, ay, c, fc | ((lc - fc - 1) << 30), rs0, rs1);
}

__global__ __launch_bounds__(kBlock) void k_dtree_level(int l, const DevScalars* __restrict__ sc,
                                                        const uint32_t* __restrict__ cursor,
                                                        Node* __restrict__ nodes,
                                                        CellF* __restrict__ c32,
                                                        double2* __restrict__ nsum) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint32_t m = sc->level_size[l];
    if (t >= m) return;
    dtree_inner(l, sc, cursor, nodes, c32, nsum, (uint32_t)t, m, cell_scale(sc->s[0]),
                cell_scale(sc->s[1]));
}

// levels top..0 in one block (a level l holds at most 4^l cells)
__global__ __launch_bounds__(kTopThreads) void k_dtree_top(int top,
                                                           const DevScalars* __restrict__ sc,
                                                           const uint32_t* __restrict__ cursor,
                                                           Node* __restrict__ nodes,
                                                           CellF* __restrict__ c32,
                                                           double2* __restrict__ nsum) {
    const float rs0 = cell_scale(sc->s[0]), rs1 = cell_scale(sc->s[1]);
    for (int l = top; l >= 0; l--) {
        const uint32_t m = sc->level_size[l];
        for (uint32_t t = threadIdx.x; t < m; t += kTopThreads)
            dtree_inner(l, sc, cursor, nodes, c32, nsum, t, m, rs0, rs1);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_export_dtree(const Node* __restrict__ nodes,
                                                         const double2* __restrict__ nsum,
                                                         const uint64_t* __restrict__ keys,
                                                         const DevScalars* __restrict__ sc,
                                                         uint64_t* __restrict__ prefix,
                                                         uint32_t* __restrict__ count,
                                                         double* __restrict__ sum) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= sc->n_nodes) return;
    const Node nd = nodes[g];
    const int sh = 2 * (kDLevels - (int)nd.level);
    if (prefix) prefix[g] = sh >= 64 ? 0ull : (keys[nd.start] >> sh);
    if (count) count[g] = nd.count;
    if (sum) {
        sum[2 * g] = nsum[g].x;
        sum[2 * g + 1] = nsum[g].y;
    }
}

}  // namespace

hipError_t run_snap_dtree(pixelsne_ctx* c) {
    TreeBufs& tb = c->tb;
    if (fp64(c))
        k_snap64<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const double*)c->zh, (double*)c->z, tb.key64[0], tb.idx[0], c->sc, c->n, c->r, c->L);
    else
        k_snap64<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            (const float*)c->zh, (float*)c->z, tb.key64[0], tb.idx[0], c->sc, c->n, c->r, c->L);
    return hipGetLastError();
}

hipError_t run_sort_dtree(pixelsne_ctx* c) {
    TreeBufs& tb = c->tb;
    int cur = 0;
    for (int p = 0; p < 8; p++) {
        const int shift = 8 * p;
        k_rs_hist64<<<dim3((unsigned)tb.sort_blocks), kBlock, 0, c->stream>>>(
            tb.key64[cur], c->n, shift, tb.hist, tb.sort_blocks);
        hipError_t e = run_rows_scan(tb.hist, 256, tb.sort_blocks, tb.dtot, c->stream);
        if (e != hipSuccess) return e;
        k_rs_scatter64<<<dim3((unsigned)tb.sort_blocks), kBlock, 0, c->stream>>>(
            tb.key64[cur], p == 0 ? nullptr : tb.idx[cur], tb.key64[cur ^ 1], tb.idx[cur ^ 1],
            c->n, shift, tb.hist, tb.dtot, tb.sort_blocks);
        cur ^= 1;
    }
    tb.sorted = cur;
    return hipGetLastError();
}

hipError_t run_tree_dtree(pixelsne_ctx* c) {
    TreeBufs& tb = c->tb;
    const uint64_t* keys = tb.key64[tb.sorted];
    const uint32_t* perm = tb.idx[tb.sorted];
    k_dtree_count<<<dim3((unsigned)tb.tree_blocks), kBlock, 0, c->stream>>>(
        keys, c->n, tb.lvl_cnt, tb.tree_blocks);
    hipError_t e = run_rows_scan(tb.lvl_cnt, kDLevels + 1, tb.tree_blocks, tb.ltot, c->stream);
    if (e != hipSuccess) return e;
    if (fp64(c)) {
        k_dtree_nodes<double><<<dim3((unsigned)tb.tree_blocks), kBlock, 0, c->stream>>>(
            keys, perm, (const double*)c->z, c->n, tb.lvl_cnt, tb.tree_blocks, tb.ltot, c->sc,
            tb.nodes, tb.cursor, tb.leaf_of, (double*)tb.zs);
        k_dtree_leaves<double><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            keys, (const double*)tb.zs, c->n, tb.leaf_of, tb.nodes, tb.cells32, tb.nsum, c->sc);
    } else {
        k_dtree_nodes<float><<<dim3((unsigned)tb.tree_blocks), kBlock, 0, c->stream>>>(
            keys, perm, (const float*)c->z, c->n, tb.lvl_cnt, tb.tree_blocks, tb.ltot, c->sc,
            tb.nodes, tb.cursor, tb.leaf_of, (float*)tb.zs);
        k_dtree_leaves<float><<<grid_for(c->n), kBlock, 0, c->stream>>>(
            keys, (const float*)tb.zs, c->n, tb.leaf_of, tb.nodes, tb.cells32, tb.nsum, c->sc);
    }
    for (int l = kDLevels - 1; l > kTopLevel; l--) {
        const int64_t cap = l < 31 ? (int64_t)1 << (2 * l) : c->n;
        k_dtree_level<<<grid_for(cap < c->n ? cap : c->n), kBlock, 0, c->stream>>>(
            l, c->sc, tb.cursor, tb.nodes, tb.cells32, tb.nsum);
    }
    k_dtree_top<<<1, kTopThreads, 0, c->stream>>>(kTopLevel, c->sc, tb.cursor, tb.nodes,
                                                  tb.cells32, tb.nsum);
    return hipGetLastError();
}

hipError_t run_export_dtree(const pixelsne_ctx* c, uint64_t* keys, uint32_t* perm,
                            uint64_t* prefix, uint32_t* count, double* sum) {
    const TreeBufs& tb = c->tb;
    hipError_t e = hipSuccess;
    if (keys)
        e = hipMemcpyAsync(keys, tb.key64[tb.sorted], (size_t)c->n * 8, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess && perm) e = run_map_perm(c, tb.idx[tb.sorted], perm);
    if (e != hipSuccess) return e;
    if (prefix || count || sum)
        k_export_dtree<<<grid_for(tb.max_nodes), kBlock, 0, c->stream>>>(
            tb.nodes, tb.nsum, tb.key64[tb.sorted], c->sc, prefix, count, sum);
    return hipGetLastError();
}

}  // namespace psne
