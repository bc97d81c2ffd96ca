// PixelSNE in three dimensions on gfx950 (declared in include/pixelsne.h).
//
// Section 1 notes that the method carries over to 3-D embeddings.  The screen
// becomes a cube of r^3 voxels and the P-Quadtree an octree of fixed depth
// L = log2 r (L <= 10) with single-voxel leaves; every per-axis step of the
// 2-D path (Eq. 1-2 snapping, Eq. 11 opening test, Eq. 12-13 scale factors,
// the Section 4.2 screen scaling) runs over three axes.  Everything is FP64.
//
// One iteration, on the context's stream:
//   keys      voxel of each point and its 30-bit Morton key (x, y, z in bits
//             3b, 3b+1, 3b+2)
//   sort      stable radix sort of (key, index) on 3L bits (shared with the
//             2-D path)
//   tree      cells of every level numbered from the sorted keys (a cell of
//             level l = a run of equal key >> 3(L - l)); leaf sums by a
//             segmented scan per wavefront and the pieces of each leaf, inner
//             sums from the <= 8 children, one launch per level
//   traverse  the 64 points of a wavefront walk the union of their paths
//             depth first without a stack: children are consecutive cells,
//             so after a cell the wave moves to the next sibling or climbs
//             to the parent
//   zsum      Z = sum of the per-point terms (fixed order)
//   attract   one wavefront per row of P
//   update    gains / momentum step and per-block min / max of z + u
//   finalize  gamma_d = max - min + eps per axis, s_d *= gamma_d / r
//   rescale   z = r (zh - min) / gamma, u *= r / gamma
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "ctx.h"

namespace psne {

constexpr int kL3Max = 10;                       // r <= 1024: 3L <= 30 key bits
constexpr int kLevels3 = kL3Max + 1;
constexpr int kChildBits3 = 29;                  // first child | (children - 1) << 29
constexpr uint32_t kChildMask3 = (1u << kChildBits3) - 1u;
constexpr int64_t kMaxN3 = (int64_t)1 << 25;     // cells <= 11 n < 2^29

struct Scalars3 {
    double s[3];        // y units per voxel, per axis
    double lo[3];       // per-axis minimum of z + u of the last update
    double gamma[3];    // max - min + eps of the last update
    double Z;           // Barnes-Hut normaliser of the last gradient
    int32_t nonfinite;
    int32_t pad;
    int64_t n_nodes;
    uint32_t level_size[kLevels3];
    uint32_t level_base[kLevels3 + 1];
};

// One octree cell as the traversal reads it (32 bytes): centre of mass (Eq. 8),
// number of points, and the first child | (children - 1) << 29; 0 for a leaf.
struct alignas(32) Node3 {
    double cx, cy, cz;
    uint32_t count;
    uint32_t child;
};

}  // namespace psne

struct pixelsne3_ctx {
    int64_t n = 0, nnz = 0;
    int32_t r = 0, L = 0, k = 0;
    int32_t t = 0;                          // iterations done
    pixelsne_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool poisoned = false;

    int64_t* row_ptr = nullptr;             // P in CSR, caller numbering
    uint32_t* col = nullptr;
    double* val = nullptr;

    double* z = nullptr;                    // [n][3] voxel frame, 0 <= z < r
    double* zh = nullptr;                   // [n][3] z + u before the scaling
    double* u = nullptr;
    double* g = nullptr;
    double* A = nullptr;
    double* R = nullptr;
    double* Zi = nullptr;                   // [n]
    double* zpart = nullptr;
    int64_t zpart_n = 0;
    double* mm_part = nullptr;              // [mm_n][6] per-block min / max
    int64_t mm_n = 0;
    psne::Scalars3* sc = nullptr;

    uint32_t* key[2] = {nullptr, nullptr};
    uint32_t* idx[2] = {nullptr, nullptr};
    int sorted = 0;
    uint32_t* hist = nullptr;
    uint32_t* dtot = nullptr;
    uint32_t* lvl_cnt = nullptr;            // [L + 1][tree_blocks]
    uint32_t* ltot = nullptr;
    int64_t tree_blocks = 0;
    int64_t max_nodes = 0;
    psne::Node3* nodes = nullptr;
    double* nsum = nullptr;                 // [max_nodes][3] coordinate sums
    uint32_t* nstart = nullptr;             // first sorted position of each cell
    uint32_t* fchild = nullptr;             // first child of each inner cell
    uint32_t* parent = nullptr;
    uint32_t* leaf_of = nullptr;            // [n] leaf of each sorted position
    double* zs = nullptr;                   // [n][3] positions in sorted order
    double* zscan = nullptr;                // [n][3] per-wave segmented leaf scan
    bool have_tree = false;

    std::vector<void*> allocs;
};

namespace psne {
namespace {

constexpr int kBlock = 256;
constexpr int64_t kUpdateBlocksMax = 2048;

inline dim3 grid_for(int64_t n) { return dim3((unsigned)ceil_div(n > 0 ? n : 1, kBlock)); }
inline int64_t update_blocks(int64_t n) {
    const int64_t b = ceil_div(n, kBlock);
    return b < kUpdateBlocksMax ? b : kUpdateBlocksMax;
}

// the bits of a 10-bit value spread to every third bit
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t voxel(double z, int r) {
    const double f = floor(z);
    if (!(f >= 0.0)) return 0u;
    if (f > (double)(r - 1)) return (uint32_t)(r - 1);
    return (uint32_t)f;
}

__device__ __forceinline__ double mul_nc3(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// b1 dx^2 + b2 dy^2 + b3 dz^2 as ((b1 dx) dx + (b2 dy) dy) + (b3 dz) dz, every
// operation rounded separately, so the opening decision is the FP64 one
__device__ __forceinline__ double dist3(double b0, double b1, double b2, double dx, double dy,
                                       double dz) {
#pragma clang fp contract(off)
    const double a = (b0 * dx) * dx;
    const double b = (b1 * dy) * dy;
    const double c = (b2 * dz) * dz;
    return (a + b) + c;
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k3_keys(const double* __restrict__ z, int64_t n, int r,
                                                  uint32_t* __restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t vx = voxel(z[3 * i], r), vy = voxel(z[3 * i + 1], r),
                   vz = voxel(z[3 * i + 2], r);
    key[i] = spread3(vx) | (spread3(vy) << 1) | (spread3(vz) << 2);
}

// ---------------------------------------------------------------------------
// tree: cells numbered level by level, each level ascending by prefix
// ---------------------------------------------------------------------------
// first level at which sorted position s opens a cell (s = 0: every level;
// a key equal to the previous one: none, L + 1)
__device__ __forceinline__ int first_new_level3(const uint32_t* __restrict__ keys, int64_t s,
                                                int L) {
    if (s == 0) return 0;
    const uint32_t x = keys[s] ^ keys[s - 1];
    if (x == 0) return L + 1;
    const int hb = 31 - __clz(x);
    return L - hb / 3;
}

__global__ __launch_bounds__(kBlock) void k3_tree_count(const uint32_t* __restrict__ keys,
                                                        int64_t n, int L,
                                                        uint32_t* __restrict__ cnt, int64_t nb) {
    __shared__ uint32_t wc[4][kLevels3];
    const int t = threadIdx.x, w = t >> 6;
    const int64_t s = (int64_t)blockIdx.x * kBlock + t;
    const int l0 = s < n ? first_new_level3(keys, s, L) : L + 1;
    for (int l = 0; l <= L; l++) {
        const uint64_t b = ballot64(l0 <= l);
        if (lane_id() == 0) wc[w][l] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (t <= L) cnt[(int64_t)t * nb + blockIdx.x] = wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
}

// For every level, the rank of the cell holding sorted position s; positions
// that open a cell record its start, first child and parent.
__global__ __launch_bounds__(kBlock) void k3_tree_nodes(
    const uint32_t* __restrict__ keys, int64_t n, int L, const uint32_t* __restrict__ off,
    int64_t nb, const uint32_t* __restrict__ ltot, Scalars3* __restrict__ sc,
    uint32_t* __restrict__ nstart, uint32_t* __restrict__ fchild, uint32_t* __restrict__ parent,
    uint32_t* __restrict__ leaf_of) {
    __shared__ uint32_t wc[4][kLevels3];
    __shared__ uint32_t lbase[kLevels3 + 1];
    const int t = threadIdx.x, w = t >> 6;
    if (t == 0) {
        uint32_t b = 0;
        for (int l = 0; l <= L; l++) {
            lbase[l] = b;
            b += ltot[l];
        }
        lbase[L + 1] = b;
        if (blockIdx.x == 0) {
            for (int l = 0; l <= L; l++) {
                sc->level_size[l] = ltot[l];
                sc->level_base[l] = lbase[l];
            }
            sc->level_base[L + 1] = b;
            sc->n_nodes = b;
        }
    }
    const int64_t s = (int64_t)blockIdx.x * kBlock + t;
    const bool valid = s < n;
    const int l0 = valid ? first_new_level3(keys, s, L) : L + 1;
    for (int l = 0; l <= L; l++) {
        const uint64_t b = ballot64(l0 <= l);
        if (lane_id() == 0) wc[w][l] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    const uint64_t le = lanemask_lt() | (1ull << lane_id());
    uint32_t cell[kLevels3];
#pragma unroll
    for (int l = 0; l < kLevels3; l++) {
        if (l <= L) {
            const uint64_t b = ballot64(l0 <= l);
            uint32_t rk = off[(int64_t)l * nb + blockIdx.x] + (uint32_t)__popcll(b & le);
            for (int q = 0; q < w; q++) rk += wc[q][l];
            cell[l] = lbase[l] + rk - 1;
        } else {
            cell[l] = 0;
        }
    }
    if (!valid) return;
    leaf_of[s] = cell[L];
#pragma unroll
    for (int l = 0; l < kLevels3; l++) {
        if (l <= L && l0 <= l) {
            const uint32_t g = cell[l];
            nstart[g] = (uint32_t)s;
            fchild[g] = l < L ? cell[l < L ? l + 1 : L] : 0u;
            parent[g] = l > 0 ? cell[l > 0 ? l - 1 : 0] : 0u;
        }
    }
}

__device__ __forceinline__ void write_cell3(Node3* __restrict__ nodes, double* __restrict__ nsum,
                                            uint32_t g, double sx, double sy, double sz,
                                            uint32_t count, uint32_t child) {
    const double m = (double)count;
    nodes[g] = Node3{sx / m, sy / m, sz / m, count, child};
    nsum[3 * (int64_t)g] = sx;
    nsum[3 * (int64_t)g + 1] = sy;
    nsum[3 * (int64_t)g + 2] = sz;
}

// Leaf sums, part 1 (one thread per sorted position): gather the point into
// sorted order (zs) and run a segmented inclusive scan over each wave's 64
// positions, segments = leaves (runs of equal leaf index), fixed shuffle
// pattern.  zscan[p] then holds the sum of the positions of p's leaf from
// max(leaf start, wave start) to p.
__global__ __launch_bounds__(kBlock) void k3_leaf_scan(const uint32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ leaf_of,
                                                       const double* __restrict__ z, int64_t n,
                                                       double* __restrict__ zs,
                                                       double* __restrict__ zscan) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = p < n;
    const int lane = lane_id();
    double v[3] = {0.0, 0.0, 0.0};
    uint32_t leaf = 0xFFFFFFFFu;
    if (valid) {
        const int64_t i = perm[p];
        for (int d = 0; d < 3; d++) v[d] = z[3 * i + d];
        leaf = leaf_of[p];
        for (int d = 0; d < 3; d++) zs[3 * p + d] = v[d];
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t lu = __shfl_up(leaf, o, kWave);
        double u[3];
        for (int d = 0; d < 3; d++) u[d] = __shfl_up(v[d], o, kWave);
        if (lane >= o && lu == leaf)
            for (int d = 0; d < 3; d++) v[d] += u[d];
    }
    if (valid)
        for (int d = 0; d < 3; d++) zscan[3 * p + d] = v[d];
}

// Leaf sums, part 2 (one thread per leaf): the piece in the wave of the
// leaf's first position, the whole waves inside the leaf, and the piece in
// the wave of its last position.
__global__ __launch_bounds__(kBlock) void k3_leaves(const double* __restrict__ zscan, int64_t n,
                                                    int L, const Scalars3* __restrict__ sc,
                                                    const uint32_t* __restrict__ nstart,
                                                    Node3* __restrict__ nodes,
                                                    double* __restrict__ nsum) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (int64_t)sc->level_size[L]) return;
    const uint32_t g = sc->level_base[L] + (uint32_t)q;
    const int64_t a = nstart[g];
    const int64_t e = g + 1 < sc->level_base[L + 1] ? (int64_t)nstart[g + 1] : n;
    const int64_t wa = a / kWave, wb = (e - 1) / kWave;
    double sm[3];
    for (int d = 0; d < 3; d++) sm[d] = zscan[3 * (e - 1) + d];
    if (wa < wb) {
        for (int d = 0; d < 3; d++) sm[d] += zscan[3 * (wa * kWave + kWave - 1) + d];
        for (int64_t w = wa + 1; w < wb; w++)
            for (int d = 0; d < 3; d++) sm[d] += zscan[3 * (w * kWave + kWave - 1) + d];
    }
    write_cell3(nodes, nsum, g, sm[0], sm[1], sm[2], (uint32_t)(e - a), 0u);
}

// inner cells of level l: the sums of their (consecutive) children
__global__ __launch_bounds__(kBlock) void k3_inner(int l, const Scalars3* __restrict__ sc,
                                                   const uint32_t* __restrict__ fchild,
                                                   Node3* __restrict__ nodes,
                                                   double* __restrict__ nsum) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (int64_t)sc->level_size[l]) return;
    const uint32_t g = sc->level_base[l] + (uint32_t)q;
    const uint32_t c0 = fchild[g];
    const uint32_t c1 = g + 1 < sc->level_base[l + 1] ? fchild[g + 1] : sc->level_base[l + 2];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    uint32_t cnt = 0;
    for (uint32_t c = c0; c < c1; c++) {
        sx += nsum[3 * (int64_t)c];
        sy += nsum[3 * (int64_t)c + 1];
        sz += nsum[3 * (int64_t)c + 2];
        cnt += nodes[c].count;
    }
    write_cell3(nodes, nsum, g, sx, sy, sz, cnt, c0 | ((c1 - c0 - 1u) << kChildBits3));
}

// ---------------------------------------------------------------------------
// Barnes-Hut traversal (Eq. 5 second term, Eq. 11, Eq. 12 in three axes)
// ---------------------------------------------------------------------------
// A leaf is always used; the leaf holding the point itself counts its other
// points only, at their mean.  An inner cell of side w is used when
// w^2 (b1 + b2 + b3) < theta^2 d^2, else its children are visited in order.
//
// The 64 points of a wavefront (neighbours in Morton order) walk the union of
// their walks together: the wave steps through cells in depth-first order
// and enters a cell's children when any of its lanes opens the cell.  A lane
// takes part in a cell only if it opened every ancestor: `mark` holds the
// level of the last cell the lane used (or skipped), and the lane sits out
// every cell deeper than that until the wave returns to that level.  The
// cell address is the same for the whole wave, so cells arrive through
// scalar loads, and each lane's sums run in the order of its own walk.
__global__ __launch_bounds__(kBlock) void k3_traverse(
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ leaf_of,
    const double* __restrict__ zs, const Node3* __restrict__ nodes,
    const double* __restrict__ nsum, const uint32_t* __restrict__ parent,
    const Scalars3* __restrict__ sc, int64_t n, int L, double th2, double* __restrict__ R,
    double* __restrict__ Zi, uint32_t* __restrict__ visits) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = s < n;
    const int64_t i = valid ? (int64_t)perm[s] : 0;
    const uint32_t own = valid ? leaf_of[s] : 0xFFFFFFFFu;
    const double b0 = sc->s[0] * sc->s[0], b1 = sc->s[1] * sc->s[1], b2 = sc->s[2] * sc->s[2];
    double bs;
    {
#pragma clang fp contract(off)
        bs = (b0 + b1) + b2;
    }
    const double x = valid ? zs[3 * s] : 0.0, y = valid ? zs[3 * s + 1] : 0.0,
                 w3 = valid ? zs[3 * s + 2] : 0.0;
    double rx = 0.0, ry = 0.0, rz = 0.0, zacc = 0.0;
    uint32_t nv = 0;
    int mark = valid ? 0x7FFFFFFF : -1;
    uint32_t g = 0;
    int lvl = 0;
    for (;;) {
        const Node3 nd = nodes[g];
        bool open = false;
        if (lvl <= mark) {
            nv++;
            bool use = true;
            double m = (double)nd.count, cx = nd.cx, cy = nd.cy, cz = nd.cz;
            if (nd.child == 0u) {
                if (g == own) {
                    m -= 1.0;
                    if (m > 0.0) {
                        cx = (nsum[3 * (int64_t)g] - x) / m;
                        cy = (nsum[3 * (int64_t)g + 1] - y) / m;
                        cz = (nsum[3 * (int64_t)g + 2] - w3) / m;
                    } else {
                        use = false;
                    }
                }
            } else {
                const double d2 = dist3(b0, b1, b2, x - cx, y - cy, w3 - cz);
                const double wc = (double)(1u << (L - lvl));
                if (!(mul_nc3(mul_nc3(wc, wc), bs) < mul_nc3(th2, d2))) {
                    use = false;
                    open = true;
                }
            }
            if (use) {
                const double dx = x - cx, dy = y - cy, dz = w3 - cz;
                const double q = rcp_nr(1.0 + dist3(b0, b1, b2, dx, dy, dz));
                const double mq = m * q;
                zacc += mq;
                const double f = mq * q;
                rx += f * dx;
                ry += f * dy;
                rz += f * dz;
            }
            mark = open ? 0x7FFFFFFF : lvl;
        }
        if (ballot64(open)) {
            g = nd.child & kChildMask3;
            lvl++;
            continue;
        }
        // the next sibling, climbing while the cell is the last of its parent
        bool done = true;
        while (g != 0u) {
            const uint32_t p = parent[g];
            const uint32_t pc = nodes[p].child;
            if (g < (pc & kChildMask3) + (pc >> kChildBits3)) {
                g++;
                done = false;
                break;
            }
            g = p;
            lvl--;
        }
        if (done) break;
    }
    if (!valid) return;
    R[3 * i] = rx;
    R[3 * i + 1] = ry;
    R[3 * i + 2] = rz;
    Zi[i] = zacc;
    if (visits) visits[i] = nv;
}

__global__ __launch_bounds__(kBlock) void k3_zpart(const double* __restrict__ Zi, int64_t n,
                                                   double* __restrict__ part) {
    __shared__ double red[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    red[threadIdx.x] = i < n ? Zi[i] : 0.0;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k3_zfinal(const double* __restrict__ part, int64_t m,
                                                    Scalars3* __restrict__ sc) {
    __shared__ double red[kBlock];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kBlock) a += part[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->Z = red[0];
}

// ---------------------------------------------------------------------------
// attraction A_i = sum_j p_ij w_ij (z_i - z_j) (Eq. 5 first term, Eq. 12)
// ---------------------------------------------------------------------------
// Rows are taken in the Morton order of their points (perm), so that waves
// running at the same time gather the positions of nearby points, whose
// neighbours largely coincide.
__global__ __launch_bounds__(kBlock) void k3_attract(const int64_t* __restrict__ rp,
                                                     const uint32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ z,
                                                     const uint32_t* __restrict__ perm,
                                                     const Scalars3* __restrict__ sc, int64_t n,
                                                     double* __restrict__ A) {
    const int lane = lane_id();
    const int64_t wv = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    if (wv >= n) return;
    const int64_t row = perm[wv];
    const double b0 = sc->s[0] * sc->s[0], b1 = sc->s[1] * sc->s[1], b2 = sc->s[2] * sc->s[2];
    const double x = z[3 * row], y = z[3 * row + 1], w3 = z[3 * row + 2];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t e = rp[row] + lane; e < rp[row + 1]; e += kWave) {
        const int64_t j = col[e];
        const double dx = x - z[3 * j], dy = y - z[3 * j + 1], dz = w3 - z[3 * j + 2];
        const double pq = val[e] * rcp_nr(1.0 + dist3(b0, b1, b2, dx, dy, dz));
        ax += pq * dx;
        ay += pq * dy;
        az += pq * dz;
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    az = wave_sum(az);
    if (lane == 0) {
        A[3 * row] = ax;
        A[3 * row + 1] = ay;
        A[3 * row + 2] = az;
    }
}

// B = alpha A - R / Z
__global__ __launch_bounds__(kBlock) void k3_bracket(const double* __restrict__ A,
                                                     const double* __restrict__ R,
                                                     const Scalars3* __restrict__ sc, int64_t m,
                                                     double alpha, double* __restrict__ B) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < m) B[e] = alpha * A[e] - R[e] / sc->Z;
}

// ---------------------------------------------------------------------------
// update: gains, momentum, zh = z + u, per-block min / max of zh
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sgn3(double v) { return (v > 0.0) - (v < 0.0); }

__device__ __forceinline__ void block_minmax6(double* v, double* __restrict__ out) {
    __shared__ double red[4][6];
    const int lane = lane_id(), w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; k++) v[k] = k < 3 ? wave_min(v[k]) : wave_max(v[k]);
    if (lane == 0)
        for (int k = 0; k < 6; k++) red[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double a = red[0][k];
        for (int q = 1; q < 4; q++) a = k < 3 ? fmin(a, red[q][k]) : fmax(a, red[q][k]);
        out[6 * (int64_t)blockIdx.x + k] = a;
    }
}

__global__ __launch_bounds__(kBlock) void k3_update(
    const double* __restrict__ A, const double* __restrict__ R, const double* __restrict__ z,
    double* __restrict__ u, double* __restrict__ g, double* __restrict__ zh,
    Scalars3* __restrict__ sc, int64_t n, double alpha, double mu, double eta, double gmin,
    double* __restrict__ mm_part) {
    const double Z = sc->Z;
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const int64_t e = 3 * i + d;
            const double b = alpha * A[e] - R[e] / Z;
            const double ue = u[e];
            double gn = sgn3(b) != sgn3(ue) ? g[e] + 0.2 : g[e] * 0.8;
            gn = gn < gmin ? gmin : gn;
            const double un = mu * ue - eta * gn * b;
            const double h = z[e] + un;
            g[e] = gn;
            u[e] = un;
            zh[e] = h;
            if (!isfinite(h)) bad = true;
            v[d] = fmin(v[d], h);
            v[3 + d] = fmax(v[3 + d], h);
        }
    }
    if (ballot64(bad) && lane_id() == 0) atomicOr(&sc->nonfinite, 1);
    block_minmax6(v, mm_part);
}

__global__ __launch_bounds__(kBlock) void k3_minmax(const double* __restrict__ zh, int64_t n,
                                                    double* __restrict__ mm_part) {
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
#pragma unroll
        for (int d = 0; d < 3; d++) {
            v[d] = fmin(v[d], zh[3 * i + d]);
            v[3 + d] = fmax(v[3 + d], zh[3 * i + d]);
        }
    block_minmax6(v, mm_part);
}

// screen-driven scaling of each axis (Section 4.2): gamma = max - min + eps,
// s *= gamma / r
__global__ __launch_bounds__(kBlock) void k3_finalize(const double* __restrict__ mm_part,
                                                      int64_t m, Scalars3* __restrict__ sc, int r,
                                                      double eps) {
    __shared__ double red[6][kBlock];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = threadIdx.x; i < m; i += kBlock)
        for (int k = 0; k < 6; k++)
            v[k] = k < 3 ? fmin(v[k], mm_part[6 * i + k]) : fmax(v[k], mm_part[6 * i + k]);
    for (int k = 0; k < 6; k++) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const int a = threadIdx.x, b = threadIdx.x + o;
            for (int k = 0; k < 6; k++)
                red[k][a] = k < 3 ? fmin(red[k][a], red[k][b]) : fmax(red[k][a], red[k][b]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int d = 0; d < 3; d++) {
            const double lo = red[d][0], gam = red[3 + d][0] - lo + eps;
            sc->lo[d] = lo;
            sc->gamma[d] = gam;
            sc->s[d] *= gam / (double)r;
            if (!isfinite(gam)) sc->nonfinite = 1;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k3_rescale(const double* __restrict__ zh,
                                                     double* __restrict__ z,
                                                     double* __restrict__ u,
                                                     const Scalars3* __restrict__ sc, int64_t m,
                                                     int r) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const int d = (int)(e % 3);
    const double gam = sc->gamma[d];
    z[e] = (double)r * (zh[e] - sc->lo[d]) / gam;
    u[e] *= (double)r / gam;
}

// initial state: Y (y frame) or N(0, sigma^2 I) from the seed (Box-Muller on
// SplitMix64 uniforms, two draws per coordinate)
__global__ __launch_bounds__(kBlock) void k3_init(const double* __restrict__ Y,
                                                  double* __restrict__ zh, double* __restrict__ u,
                                                  double* __restrict__ g, int64_t m,
                                                  uint64_t seed, double sigma) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    double y;
    if (Y) {
        y = Y[e];
    } else {
        const uint64_t a = splitmix64(seed ^ (2ull * (uint64_t)e));
        const uint64_t b = splitmix64(seed ^ (2ull * (uint64_t)e + 1ull));
        const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53;
        const double u2 = ((double)(b >> 11) + 0.5) * 0x1.0p-53;
        y = sigma * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    }
    zh[e] = y;
    u[e] = 0.0;
    g[e] = 1.0;
}

__global__ __launch_bounds__(kBlock) void k3_set_state(const double* __restrict__ uin,
                                                       const double* __restrict__ gin,
                                                       double* __restrict__ u,
                                                       double* __restrict__ g, int64_t m) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    u[e] = uin ? uin[e] : 0.0;
    g[e] = gin ? gin[e] : 1.0;
}

__global__ __launch_bounds__(kBlock) void k3_get_y(const double* __restrict__ z,
                                                   const Scalars3* __restrict__ sc, int64_t m,
                                                   int r, int frame, void* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const int d = (int)(e % 3);
    if (frame == PSNE_FRAME_SCREEN)
        reinterpret_cast<int32_t*>(out)[e] = (int32_t)voxel(z[e], r);
    else if (frame == PSNE_FRAME_Y)
        reinterpret_cast<double*>(out)[e] = sc->s[d] * z[e];
    else
        reinterpret_cast<double*>(out)[e] = z[e];
}

__global__ __launch_bounds__(kBlock) void k3_export(const Node3* __restrict__ nodes,
                                                    const double* __restrict__ nsum,
                                                    const uint32_t* __restrict__ nstart,
                                                    const uint32_t* __restrict__ keys,
                                                    const Scalars3* __restrict__ sc, int L,
                                                    uint32_t* __restrict__ prefix,
                                                    uint32_t* __restrict__ count,
                                                    double* __restrict__ sum) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= sc->n_nodes) return;
    int l = 0;
    while (l < L && (int64_t)sc->level_base[l + 1] <= g) l++;
    if (prefix) prefix[g] = keys[nstart[g]] >> (3 * (L - l));
    if (count) count[g] = nodes[g].count;
    if (sum)
        for (int d = 0; d < 3; d++) sum[3 * g + d] = nsum[3 * g + d];
}

// ---------------------------------------------------------------------------
// KL (Eq. 4) with the exact normaliser, three axes
// ---------------------------------------------------------------------------
struct F3 { float x, y, z; };

__global__ __launch_bounds__(kBlock) void k3_kl_z(const double* __restrict__ z,
                                                  const Scalars3* __restrict__ sc, int64_t n,
                                                  double* __restrict__ part) {
    __shared__ F3 tile[kBlock];
    __shared__ double red[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const float b0 = (float)(sc->s[0] * sc->s[0]), b1 = (float)(sc->s[1] * sc->s[1]),
                b2 = (float)(sc->s[2] * sc->s[2]);
    F3 zi{0.f, 0.f, 0.f};
    if (i < n) zi = F3{(float)z[3 * i], (float)z[3 * i + 1], (float)z[3 * i + 2]};
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kBlock) {
        __syncthreads();
        const int64_t j = j0 + threadIdx.x;
        if (j < n) tile[threadIdx.x] = F3{(float)z[3 * j], (float)z[3 * j + 1], (float)z[3 * j + 2]};
        __syncthreads();
        const int m = n - j0 < kBlock ? (int)(n - j0) : kBlock;
        float sacc = 0.f;
        for (int q = 0; q < m; q++) {
            const float dx = zi.x - tile[q].x, dy = zi.y - tile[q].y, dz = zi.z - tile[q].z;
            const float w = __builtin_amdgcn_rcpf(1.0f + b0 * dx * dx + b1 * dy * dy + b2 * dz * dz);
            sacc += (j0 + q == i) ? 0.f : w;
        }
        if (i < n) acc += (double)sacc;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k3_kl_p(const int64_t* __restrict__ rp,
                                                  const uint32_t* __restrict__ col,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ z,
                                                  const Scalars3* __restrict__ sc, int64_t n,
                                                  double* __restrict__ part) {
    __shared__ double red[4][2];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * 4 + w, nw = (int64_t)gridDim.x * 4;
    const double b0 = sc->s[0] * sc->s[0], b1 = sc->s[1] * sc->s[1], b2 = sc->s[2] * sc->s[2];
    double a = 0.0, ps = 0.0;
    for (int64_t i = wave; i < n; i += nw) {
        for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += kWave) {
            const double p = val[e];
            if (!(p > 0.0)) continue;
            const int64_t j = col[e];
            const double dx = z[3 * i] - z[3 * j], dy = z[3 * i + 1] - z[3 * j + 1],
                         dz = z[3 * i + 2] - z[3 * j + 2];
            a += p * log(p) + p * log(1.0 + b0 * dx * dx + b1 * dy * dy + b2 * dz * dz);
            ps += p;
        }
    }
    a = wave_sum(a);
    ps = wave_sum(ps);
    if (lane == 0) { red[w][0] = a; red[w][1] = ps; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
        part[2 * blockIdx.x + 1] = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
    }
}

__global__ __launch_bounds__(kBlock) void k3_kl_final(const double* __restrict__ part, int64_t nz,
                                                      int64_t np, double* __restrict__ out) {
    __shared__ double red[3][kBlock];
    double zs = 0.0, a = 0.0, ps = 0.0;
    for (int64_t i = threadIdx.x; i < nz; i += kBlock) zs += part[i];
    for (int64_t i = threadIdx.x; i < np; i += kBlock) {
        a += part[nz + 2 * i];
        ps += part[nz + 2 * i + 1];
    }
    red[0][threadIdx.x] = zs;
    red[1][threadIdx.x] = a;
    red[2][threadIdx.x] = ps;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 3; q++) red[q][threadIdx.x] += red[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
psne_status invalid3(const std::string& m) {
    set_error(m);
    return PSNE_E_INVAL;
}

psne_status dev_error3(pixelsne3_ctx* c, hipError_t e, const char* where) {
    if (c) c->poisoned = true;
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PSNE_E_NOMEM : PSNE_E_DEVICE;
}

psne_status usable3(const pixelsne3_ctx* c) {
    if (!c) return invalid3("null context");
    if (c->poisoned) {
        set_error("context unusable after a device error");
        return PSNE_E_STATE;
    }
    return PSNE_OK;
}

template <typename P>
hipError_t dalloc3(pixelsne3_ctx* c, P** out, size_t bytes) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
    if (e != hipSuccess) return e;
    c->allocs.push_back(p);
    *out = (P*)p;
    return hipSuccess;
}

void free3(pixelsne3_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : c->allocs) (void)hipFree(p);
    delete c;
}

psne_status check_params3(const pixelsne_params* p) {
    if (p->struct_size != sizeof(pixelsne_params))
        return invalid3("pixelsne_params.struct_size does not match this library");
    if (!(p->theta >= 0.0 && p->theta <= 0.99)) return invalid3("theta must be in [0, 0.99]");
    if (!(p->eta > 0.0) || !(p->exaggeration > 0.0))
        return invalid3("eta and exaggeration must be > 0");
    if (!(p->min_gain >= 0.0) || !(p->eps > 0.0)) return invalid3("min_gain >= 0 and eps > 0 required");
    if (p->x_dtype != PSNE_X_F32 && p->x_dtype != PSNE_X_F64 && p->x_dtype != PSNE_X_U8)
        return invalid3("unknown x_dtype");
    if (p->exag_iters < 0 || p->mom_switch < 0) return invalid3("negative schedule length");
    if (p->knn_trees < 0 || p->knn_leaf < 0 || p->knn_explore < 0)
        return invalid3("knn_trees, knn_leaf and knn_explore must be >= 0");
    if (p->precision != PSNE_FP64 || p->com_mode != PSNE_COM_MASS || p->tree != PSNE_TREE_PIXEL) {
        set_error("the 3-D path computes in FP64 with centres of mass on the voxel octree: "
                  "precision PSNE_FP64, com_mode PSNE_COM_MASS and tree PSNE_TREE_PIXEL required");
        return PSNE_E_UNSUPPORTED;
    }
    return PSNE_OK;
}

psne_status check_cube(int32_t r, int* L) {
    if (r < 2 || r > (1 << kL3Max) || (r & (r - 1))) {
        set_error("the 3-D screen side must be a power of two in [2, 1024]");
        return PSNE_E_UNSUPPORTED;
    }
    int l = 0;
    while ((1 << l) < r) l++;
    *L = l;
    return PSNE_OK;
}

pixelsne3_ctx* new3(int64_t n, int32_t r, int L, const pixelsne_params* p) {
    pixelsne3_ctx* c = new pixelsne3_ctx();
    c->n = n;
    c->r = r;
    c->L = L;
    c->prm = *p;
    c->stream = (hipStream_t)p->stream;
    (void)hipGetDevice(&c->device);
    return c;
}

hipError_t alloc3(pixelsne3_ctx* c) {
    const int64_t n = c->n;
    const size_t v3 = (size_t)n * 3 * sizeof(double);
    hipError_t e;
    double** vecs[] = {&c->z, &c->zh, &c->u, &c->g, &c->A, &c->R};
    for (double** v : vecs)
        if ((e = dalloc3(c, v, v3)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->Zi, 8 * (size_t)n)) != hipSuccess) return e;
    c->zpart_n = ceil_div(n, kBlock);
    if ((e = dalloc3(c, &c->zpart, 8 * (size_t)c->zpart_n)) != hipSuccess) return e;
    c->mm_n = update_blocks(n);
    if ((e = dalloc3(c, &c->mm_part, 6 * 8 * (size_t)c->mm_n)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->sc, sizeof(Scalars3))) != hipSuccess) return e;
    for (int h = 0; h < 2; h++) {
        if ((e = dalloc3(c, &c->key[h], 4 * (size_t)n)) != hipSuccess) return e;
        if ((e = dalloc3(c, &c->idx[h], 4 * (size_t)n)) != hipSuccess) return e;
    }
    if ((e = dalloc3(c, &c->hist, 4 * 256 * (size_t)sort_blocks_for(n))) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->dtot, 4 * 256)) != hipSuccess) return e;
    c->tree_blocks = ceil_div(n, kBlock);
    if ((e = dalloc3(c, &c->lvl_cnt, 4 * (size_t)(c->L + 1) * c->tree_blocks)) != hipSuccess)
        return e;
    if ((e = dalloc3(c, &c->ltot, 4 * (size_t)(c->L + 1))) != hipSuccess) return e;
    int64_t mx = 0;
    for (int l = 0; l <= c->L; l++) {
        const int64_t cap = (int64_t)1 << (3 * l);
        mx += cap < n ? cap : n;
    }
    c->max_nodes = mx;
    if ((e = dalloc3(c, &c->nodes, sizeof(Node3) * (size_t)mx)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->nsum, 3 * 8 * (size_t)mx)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->nstart, 4 * (size_t)mx)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->fchild, 4 * (size_t)mx)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->parent, 4 * (size_t)mx)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->leaf_of, 4 * (size_t)n)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->zs, v3)) != hipSuccess) return e;
    if ((e = dalloc3(c, &c->zscan, v3)) != hipSuccess) return e;
    return hipSuccess;
}

// per-axis scaling of zh into z (and of u), s *= gamma / r
hipError_t run_scale3(pixelsne3_ctx* c) {
    const int64_t m = 3 * c->n;
    k3_finalize<<<1, kBlock, 0, c->stream>>>(c->mm_part, c->mm_n, c->sc, c->r, c->prm.eps);
    k3_rescale<<<grid_for(m), kBlock, 0, c->stream>>>(c->zh, c->z, c->u, c->sc, m, c->r);
    return hipGetLastError();
}

hipError_t run_init3(pixelsne3_ctx* c) {
    Scalars3 h{};
    h.s[0] = h.s[1] = h.s[2] = 1.0;        // the initial frame is y itself
    hipError_t e = hipMemcpyAsync(c->sc, &h, sizeof(h), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    const int64_t m = 3 * c->n;
    k3_init<<<grid_for(m), kBlock, 0, c->stream>>>(c->prm.Y_init, c->zh, c->u, c->g, m,
                                                   c->prm.seed, c->prm.init_sigma);
    k3_minmax<<<dim3((unsigned)c->mm_n), kBlock, 0, c->stream>>>(c->zh, c->n, c->mm_part);
    return run_scale3(c);
}

// keys, sort, octree, traversal, Z and attraction at the current state
hipError_t run_forces3(pixelsne3_ctx* c, uint32_t* visits) {
    const int64_t n = c->n;
    k3_keys<<<grid_for(n), kBlock, 0, c->stream>>>(c->z, n, c->r, c->key[0]);
    hipError_t e = sort_pairs32(c->key, c->idx, n, 3 * c->L, c->hist, c->dtot, c->stream,
                                &c->sorted);
    if (e != hipSuccess) return e;
    const uint32_t* keys = c->key[c->sorted];
    const uint32_t* perm = c->idx[c->sorted];
    k3_tree_count<<<dim3((unsigned)c->tree_blocks), kBlock, 0, c->stream>>>(
        keys, n, c->L, c->lvl_cnt, c->tree_blocks);
    e = run_rows_scan(c->lvl_cnt, c->L + 1, c->tree_blocks, c->ltot, c->stream);
    if (e != hipSuccess) return e;
    k3_tree_nodes<<<dim3((unsigned)c->tree_blocks), kBlock, 0, c->stream>>>(
        keys, n, c->L, c->lvl_cnt, c->tree_blocks, c->ltot, c->sc, c->nstart, c->fchild,
        c->parent, c->leaf_of);
    k3_leaf_scan<<<grid_for(n), kBlock, 0, c->stream>>>(perm, c->leaf_of, c->z, n, c->zs,
                                                        c->zscan);
    k3_leaves<<<grid_for(n), kBlock, 0, c->stream>>>(c->zscan, n, c->L, c->sc, c->nstart,
                                                     c->nodes, c->nsum);
    for (int l = c->L - 1; l >= 0; l--) {
        const int64_t cap = (int64_t)1 << (3 * l);
        k3_inner<<<grid_for(cap < n ? cap : n), kBlock, 0, c->stream>>>(l, c->sc, c->fchild,
                                                                         c->nodes, c->nsum);
    }
    k3_traverse<<<grid_for(n), kBlock, 0, c->stream>>>(
        perm, c->leaf_of, c->zs, c->nodes, c->nsum, c->parent, c->sc, n, c->L,
        c->prm.theta * c->prm.theta, c->R, c->Zi, visits);
    k3_zpart<<<dim3((unsigned)c->zpart_n), kBlock, 0, c->stream>>>(c->Zi, n, c->zpart);
    k3_zfinal<<<1, kBlock, 0, c->stream>>>(c->zpart, c->zpart_n, c->sc);
    k3_attract<<<dim3((unsigned)ceil_div(n, kBlock / kWave)), kBlock, 0, c->stream>>>(
        c->row_ptr, c->col, c->val, c->z, perm, c->sc, n, c->A);
    c->have_tree = true;
    return hipGetLastError();
}

hipError_t run_iteration3(pixelsne3_ctx* c) {
    hipError_t e = run_forces3(c, nullptr);
    if (e != hipSuccess) return e;
    const pixelsne_params& p = c->prm;
    const double alpha = c->t < p.exag_iters ? p.exaggeration : 1.0;
    const double mu = c->t < p.mom_switch ? p.mom0 : p.mom1;
    k3_update<<<dim3((unsigned)c->mm_n), kBlock, 0, c->stream>>>(
        c->A, c->R, c->z, c->u, c->g, c->zh, c->sc, c->n, alpha, mu, p.eta, p.min_gain,
        c->mm_part);
    e = run_scale3(c);
    if (e == hipSuccess) c->t++;
    return e;
}

// state buffers and the initial embedding; P must already be in the context
psne_status finish3(pixelsne3_ctx* c) {
    hipError_t e = alloc3(c);
    if (e != hipSuccess) return dev_error3(c, e, "allocation");
    if (c->prm.Y_init && !is_device_ptr(c->prm.Y_init))
        return invalid3("Y_init must be a device pointer");
    e = run_init3(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_error3(c, e, "initial embedding");
    return PSNE_OK;
}

}  // namespace
}  // namespace psne

using namespace psne;

extern "C" {

pixelsne3_ctx* pixelsne3_init_ex(const void* X, int64_t n, int32_t D, double perplexity,
                                 int32_t r, const pixelsne_params* pin) {
    pixelsne_params p;
    if (pin) p = *pin;
    else {
        pixelsne_default_params(&p);
        p.precision = PSNE_FP64;
    }
    if (check_params3(&p) != PSNE_OK) return nullptr;
    if (n < 2 || n > kMaxN3) { invalid3("n must be in [2, 2^25]"); return nullptr; }
    if (D < 1) { invalid3("D must be >= 1"); return nullptr; }
    if (!(perplexity > 0.0) || !isfinite(perplexity)) { invalid3("perplexity must be > 0"); return nullptr; }
    const int64_t k = p.k > 0 ? p.k : (int64_t)floor(3.0 * perplexity);
    if (k < 1 || k > n - 1) { invalid3("k = floor(3 * perplexity) must be in [1, n - 1]"); return nullptr; }
    if (k > 256) { set_error("k > 256 is not supported"); return nullptr; }
    const int32_t leaf = p.knn_leaf > 0 ? p.knn_leaf : (int32_t)(2 * k + 2);
    if (p.knn_trees > 0 && leaf < 2 * k + 2) { invalid3("knn_leaf must be >= 2k + 2"); return nullptr; }
    int L;
    if (check_cube(r, &L) != PSNE_OK) return nullptr;
    if (!is_device_ptr(X)) { invalid3("X must be a device pointer"); return nullptr; }

    pixelsne3_ctx* c = new3(n, r, L, &p);
    c->k = (int32_t)k;
    int32_t* idx = nullptr;
    double *d2 = nullptr, *Pc = nullptr;
    hipError_t e = hipMalloc(&idx, sizeof(int32_t) * n * k);
    if (e == hipSuccess) e = hipMalloc(&d2, sizeof(double) * n * k);
    if (e == hipSuccess) e = hipMalloc(&Pc, sizeof(double) * n * k);
    std::string err;
    if (e == hipSuccess)
        e = p.knn_trees > 0
                ? psne::knn_approx(X, n, D, p.x_dtype, (int32_t)k, p.knn_trees, leaf,
                                   p.knn_explore, p.seed, idx, d2, c->stream, &err)
                : psne::knn(X, n, D, p.x_dtype, (int32_t)k, idx, d2, c->stream, &err);
    if (e == hipSuccess) e = psne::perplexity(d2, n, (int32_t)k, perplexity, Pc, nullptr, c->stream);
    if (e == hipSuccess)
        e = psne::symmetrize(idx, Pc, n, (int32_t)k, &c->row_ptr, &c->col, &c->val, &c->nnz,
                             c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(idx);
    (void)hipFree(d2);
    (void)hipFree(Pc);
    if (c->row_ptr) c->allocs.push_back(c->row_ptr);
    if (c->col) c->allocs.push_back(c->col);
    if (c->val) c->allocs.push_back(c->val);
    if (e != hipSuccess) {
        if (!err.empty()) set_error(err);
        else dev_error3(c, e, "building P");
        free3(c);
        return nullptr;
    }
    if (finish3(c) != PSNE_OK) { free3(c); return nullptr; }
    return c;
}

pixelsne3_ctx* pixelsne3_init_with_P(int64_t n, int64_t nnz, const int64_t* row_ptr,
                                     const int32_t* col, const double* val, int32_t r,
                                     const pixelsne_params* pin) {
    pixelsne_params p;
    if (pin) p = *pin;
    else {
        pixelsne_default_params(&p);
        p.precision = PSNE_FP64;
    }
    if (check_params3(&p) != PSNE_OK) return nullptr;
    if (n < 2 || n > kMaxN3) { invalid3("n must be in [2, 2^25]"); return nullptr; }
    if (nnz < 1) { invalid3("nnz must be >= 1"); return nullptr; }
    int L;
    if (check_cube(r, &L) != PSNE_OK) return nullptr;
    if (!is_device_ptr(row_ptr) || !is_device_ptr(col) || !is_device_ptr(val)) {
        invalid3("row_ptr, col and val must be device pointers");
        return nullptr;
    }
    pixelsne3_ctx* c = new3(n, r, L, &p);
    c->nnz = nnz;
    hipError_t e = dalloc3(c, &c->row_ptr, 8 * (size_t)(n + 1));
    if (e == hipSuccess) e = dalloc3(c, &c->col, 4 * (size_t)nnz);
    if (e == hipSuccess) e = dalloc3(c, &c->val, 8 * (size_t)nnz);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->row_ptr, row_ptr, 8 * (size_t)(n + 1), hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->col, col, 4 * (size_t)nnz, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->val, val, 8 * (size_t)nnz, hipMemcpyDeviceToDevice, c->stream);
    int64_t bad = 0;
    if (e == hipSuccess) e = check_csr(c->row_ptr, c->col, n, nnz, c->stream, &bad);
    if (e != hipSuccess) { dev_error3(c, e, "copying P"); free3(c); return nullptr; }
    if (bad) {
        invalid3("P is not a valid CSR (row_ptr from 0 to nnz, ascending; columns in [0, n) and "
                 "off the diagonal)");
        free3(c);
        return nullptr;
    }
    if (finish3(c) != PSNE_OK) { free3(c); return nullptr; }
    return c;
}

void pixelsne3_destroy(pixelsne3_ctx* c) { free3(c); }

psne_status pixelsne3_step(pixelsne3_ctx* c, int32_t n_iter) {
    psne_status st = usable3(c);
    if (st != PSNE_OK) return st;
    if (n_iter < 0) return invalid3("n_iter must be >= 0");
    for (int32_t it = 0; it < n_iter; it++) {
        hipError_t e = run_iteration3(c);
        if (e != hipSuccess) return dev_error3(c, e, "iteration");
    }
    int32_t bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, &c->sc->nonfinite, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_error3(c, e, "step");
    if (bad) {
        set_error("non-finite positions");
        return PSNE_E_NUMERIC;
    }
    return PSNE_OK;
}

psne_status pixelsne3_get_Y(const pixelsne3_ctx* c, void* out, int32_t frame) {
    psne_status st = usable3(c);
    if (st != PSNE_OK) return st;
    if (frame != PSNE_FRAME_PIXEL && frame != PSNE_FRAME_SCREEN && frame != PSNE_FRAME_Y)
        return invalid3("unknown frame");
    if (!is_device_ptr(out)) return invalid3("out must be a device pointer");
    const int64_t m = 3 * c->n;
    k3_get_y<<<grid_for(m), kBlock, 0, c->stream>>>(c->z, c->sc, m, c->r, frame, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dev_error3(const_cast<pixelsne3_ctx*>(c), e, "get_Y");
    return PSNE_OK;
}

psne_status pixelsne3_set_state(pixelsne3_ctx* c, const double* z, const double* u,
                                const double* g, const double* s, int32_t iteration) {
    psne_status st = usable3(c);
    if (st != PSNE_OK) return st;
    if (!z || !s || iteration < 0) return invalid3("z and s required, iteration >= 0");
    if (!is_device_ptr(z) || (u && !is_device_ptr(u)) || (g && !is_device_ptr(g)))
        return invalid3("z, u and g must be device pointers");
    for (int d = 0; d < 3; d++)
        if (!(s[d] > 0.0) || !isfinite(s[d])) return invalid3("s must be positive and finite");
    const int64_t m = 3 * c->n;
    hipError_t e = hipMemcpyAsync(c->z, z, 8 * (size_t)m, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) {
        k3_set_state<<<grid_for(m), kBlock, 0, c->stream>>>(u, g, c->u, c->g, m);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->sc->s, s, 3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_error3(c, e, "set_state");
    c->t = iteration;
    c->have_tree = false;
    return PSNE_OK;
}

psne_status pixelsne3_get_state(const pixelsne3_ctx* c, double* z, double* u, double* g,
                                double* s, int32_t* iteration) {
    psne_status st = usable3(c);
    if (st != PSNE_OK) return st;
    const size_t b = 8 * 3 * (size_t)c->n;
    hipError_t e = hipSuccess;
    const double* src[3] = {c->z, c->u, c->g};
    double* dst[3] = {z, u, g};
    for (int q = 0; q < 3 && e == hipSuccess; q++)
        if (dst[q]) e = hipMemcpyAsync(dst[q], src[q], b, hipMemcpyDeviceToDevice, c->stream);
    double hs[3];
    if (e == hipSuccess)
        e = hipMemcpyAsync(hs, c->sc->s, sizeof(hs), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_error3(const_cast<pixelsne3_ctx*>(c), e, "get_state");
    if (s) memcpy(s, hs, sizeof(hs));
    if (iteration) *iteration = c->t;
    return PSNE_OK;
}

psne_status pixelsne3_gradient(pixelsne3_ctx* c, double alpha, double* B, double* A, double* R,
                               double* Zi, uint32_t* visits, double* Z) {
    psne_status st = usable3(c);
    if (st != PSNE_OK) return st;
    if (!isfinite(alpha)) return invalid3("alpha must be finite");
    const int64_t m = 3 * c->n;
    hipError_t e = run_forces3(c, visits);
    if (e == hipSuccess && B) {
        k3_bracket<<<grid_for(m), kBlock, 0, c->stream>>>(c->A, c->R, c->sc, m, alpha, B);
        e = hipGetLastError();
    }
    if (e == hipSuccess && A)
        e = hipMemcpyAsync(A, c->A, 8 * (size_t)m, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && R)
        e = hipMemcpyAsync(R, c->R, 8 * (size_t)m, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && Zi)
        e = hipMemcpyAsync(Zi, c->Zi, 8 * (size_t)c->n, hipMemcpyDeviceToDevice, c->stream);
    double hz = 0.0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&hz, &c->sc->Z, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_error3(c, e, "gradient");
    if (Z) *Z = hz;
    return PSNE_OK;
}

psne_status pixelsne3_export_tree(const pixelsne3_ctx* c, int64_t* level_size, uint32_t* keys,
                                  uint32_t* perm, uint32_t* prefix, uint32_t* count,
                                  double* sum) {
    psne_status st = usable3(c);
    if (st != PSNE_OK) return st;
    if (!level_size) return invalid3("level_size required");
    if (!c->have_tree) return invalid3("no octree yet: call pixelsne3_gradient or step first");
    Scalars3 h;
    hipError_t e = hipMemcpyAsync(&h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_error3(const_cast<pixelsne3_ctx*>(c), e, "export_tree");
    for (int l = 0; l <= c->L; l++) level_size[l] = h.level_size[l];
    const uint32_t* skeys = c->key[c->sorted];
    if (keys) e = hipMemcpyAsync(keys, skeys, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && perm)
        e = hipMemcpyAsync(perm, c->idx[c->sorted], 4 * (size_t)c->n, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess && (prefix || count || sum)) {
        k3_export<<<grid_for(h.n_nodes), kBlock, 0, c->stream>>>(c->nodes, c->nsum, c->nstart,
                                                                 skeys, c->sc, c->L, prefix,
                                                                 count, sum);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_error3(const_cast<pixelsne3_ctx*>(c), e, "export_tree");
    return PSNE_OK;
}

psne_status pixelsne3_kl(const pixelsne3_ctx* c, double* kl) {
    psne_status st = usable3(c);
    if (st != PSNE_OK) return st;
    if (!kl) return invalid3("kl required");
    const int64_t nbz = ceil_div(c->n, kBlock);
    const int64_t nbp = ceil_div(c->n, 4) < 4096 ? ceil_div(c->n, 4) : 4096;
    double* part = nullptr;
    hipError_t e = hipMalloc((void**)&part, 8 * (size_t)(nbz + 2 * nbp + 3));
    if (e != hipSuccess) return dev_error3(const_cast<pixelsne3_ctx*>(c), e, "kl");
    k3_kl_z<<<dim3((unsigned)nbz), kBlock, 0, c->stream>>>(c->z, c->sc, c->n, part);
    k3_kl_p<<<dim3((unsigned)nbp), kBlock, 0, c->stream>>>(c->row_ptr, c->col, c->val, c->z,
                                                          c->sc, c->n, part + nbz);
    k3_kl_final<<<1, kBlock, 0, c->stream>>>(part, nbz, nbp, part + nbz + 2 * nbp);
    double h[3] = {0.0, 0.0, 0.0};
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, part + nbz + 2 * nbp, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(part);
    if (e != hipSuccess) return dev_error3(const_cast<pixelsne3_ctx*>(c), e, "kl");
    *kl = h[1] + h[2] * log(h[0]);
    return PSNE_OK;
}

}  // extern "C"
