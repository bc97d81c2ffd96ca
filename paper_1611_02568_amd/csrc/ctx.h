// Host-side context of the gfx950 PixelSNE library and the launchers that the
// C ABI (capi.hip) drives.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace psne {

// Device buffers of the per-iteration tree (sized once for n points).
struct TreeBufs {
    int64_t max_nodes = 0;
    uint32_t* key[2] = {nullptr, nullptr};   // radix-sort ping-pong: Morton keys
    uint32_t* idx[2] = {nullptr, nullptr};   // ... and point indices
    int sorted = 0;                          // which half holds the sorted result
    uint32_t* hist = nullptr;                // [256][sort blocks]
    uint32_t* dtot = nullptr;                // [256] digit totals of one pass
    int64_t sort_blocks = 0;
    uint32_t* lvl_cnt = nullptr;             // [levels][tree blocks], scanned in place
    uint32_t* ltot = nullptr;                // [levels] cells per level
    int64_t tree_blocks = 0;
    double2* wfirst = nullptr;               // [n / 64] per-wave partial leaf sums
    double2* wlast = nullptr;
    uint32_t* first_child = nullptr;         // [max_nodes]
    uint32_t* cell_start = nullptr;          // [max_nodes] first sorted position (pixel tree)
    Node* nodes = nullptr;                   // [max_nodes]
    CellF* cells32 = nullptr;                // [max_nodes] FP32 copy (FP32 opening test)
    double2* nsum = nullptr;                 // [max_nodes] coordinate sums (FP64)
    uint32_t* leaf_of = nullptr;             // [n] leaf cell of each sorted position
    void* zs = nullptr;                      // [n][2] positions in sorted order (state type)
    // data-driven tree only
    uint64_t* key64[2] = {nullptr, nullptr}; // 64-bit grid Morton keys (sort ping-pong)
    uint32_t* cursor = nullptr;              // [max_nodes + 1] first cell of the next level at
                                             // or after a cell's start: its children are
                                             // [cursor[g], cursor[g + 1])
};

}  // namespace psne

struct pixelsne_ctx {
    int64_t n = 0;
    int32_t r = 0, L = 0, k = 0;
    pixelsne_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool poisoned = false;

    // P in CSR, in the caller's numbering (as given or as built by the setup)
    int64_t nnz = 0;
    int64_t* row_ptr = nullptr;
    uint32_t* col = nullptr;
    void* val = nullptr;                     // state type

    // optimiser state (state type, [n][2])
    void* zh = nullptr;                      // positions before the pending screen scaling
    void* z = nullptr;                       // normalised positions (written by the snap pass)
    void* u = nullptr;
    void* g = nullptr;
    void* R = nullptr;                       // Barnes-Hut repulsion, original order
    double* Zi = nullptr;                    // per-point normaliser terms (debug output)
    double* zpart = nullptr;
    int64_t zpart_n = 0;
    double* mm_part = nullptr;               // per-block min/max of zh
    int64_t mm_n = 0;
    psne::DevScalars* sc = nullptr;
    psne::TreeBufs tb;

    // Internal order: points are renumbered by their Morton order on a
    // schedule (prm.reorder_every, prm.reorder_growth) so that the neighbours
    // of a CSR row sit close in memory.  orig[i] is the caller's index of internal point i and
    // inv its inverse.
    uint32_t* orig = nullptr;
    uint32_t* orig2 = nullptr;
    uint32_t* inv = nullptr;
    void* zh2 = nullptr;
    void* u2 = nullptr;
    void* g2 = nullptr;
    int64_t* len_tmp = nullptr;              // [n + 1]
    int64_t* scan_tmp = nullptr;
    int32_t since_reorder = 0;               // iterations since the last renumbering
    int64_t reorder_interval = 0;            // ... at which the next one is due
    int32_t scheduled_reorders = 0;
    int32_t since_reorder0 = 0;              // since_reorder at iteration 0 (schedule origin)

    // P for the attraction pass: internal rows cut into chunks of at most
    // kChunkRows consecutive rows; within a chunk the nonzeros are ordered by
    // column, in runs of 64 that are each ordered by row.
    int64_t* rp_int = nullptr;               // [n + 1] internal-order row offsets
    uint32_t* ch_row = nullptr;              // [n + 1] first internal row of each chunk
    int64_t* ch_tmp = nullptr;               // [n + 1] chunk numbering scratch
    uint32_t* pk = nullptr;                  // [nnz] internal column | row-in-chunk << 27;
                                             // FP32: [nnz][2], each word beside its value
    void* vch = nullptr;                     // FP64: [nnz] values

    // one iteration captured as a HIP graph, one per state-buffer parity
    // (renumbering swaps the state buffers with their spares)
    hipStream_t cap_stream = nullptr;

    // The attraction's row sums (A, internal order, state type [n][2]) run on
    // a second stream, forked after the snap pass or after the cells (the
    // device chooses each iteration) and joined before the update, so that the memory-bound sums share the GPU with the sort, tree
    // and the ALU-bound traversal.  side_blocks: its persistent grid, sized
    // to leave most of each CU to the traversal.  help_blocks: the grid of
    // the helper that joins the sums on the main stream after Z.
    void* A = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_cells = nullptr, ev_join = nullptr;
    int64_t side_blocks = 0;
    int64_t help_blocks = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int32_t parity = 0;
    bool graph_failed = false;

    std::vector<void*> allocs;
};

namespace psne {

void set_error(const std::string& msg);
psne_status device_error(pixelsne_ctx* c, hipError_t e, const char* where);
bool is_device_ptr(const void* p);

// iteration passes (iter.hip); each enqueues on c->stream
hipError_t run_snap(pixelsne_ctx* c);
hipError_t run_sort(pixelsne_ctx* c);
// the data-driven tree (dtree.hip): snap with 64-bit grid keys, their sort,
// and the cells; run_snap / run_sort / run_tree call these in that mode
hipError_t run_snap_dtree(pixelsne_ctx* c);
hipError_t run_sort_dtree(pixelsne_ctx* c);
hipError_t run_tree_dtree(pixelsne_ctx* c);
hipError_t run_export_dtree(const pixelsne_ctx* c, uint64_t* keys, uint32_t* perm,
                            uint64_t* prefix, uint32_t* count, double* sum);
// exclusive scan of each row of a [rows][len] uint32 array in place; row totals to tot
hipError_t run_rows_scan(uint32_t* a, int64_t rows, int64_t len, uint32_t* tot, hipStream_t s);
// stable sort of (tb.key[0], index) on the low `bits` key bits
hipError_t run_sort_bits(pixelsne_ctx* c, int bits);
// stable LSD radix sort (8-bit digits) of the pairs (key[0][i], i) on the low
// `bits` key bits; the result lands in key[*sorted], idx[*sorted].  hist holds
// 256 * sort_blocks_for(n) words, dtot 256.
int64_t sort_blocks_for(int64_t n);
hipError_t sort_pairs32(uint32_t* const key[2], uint32_t* const idx[2], int64_t n, int bits,
                        uint32_t* hist, uint32_t* dtot, hipStream_t s, int* sorted);
hipError_t run_tree(pixelsne_ctx* c);
hipError_t run_traverse(pixelsne_ctx* c, uint32_t* visits, uint32_t* used, double* Zi);
hipError_t run_zsum(pixelsne_ctx* c);
// mode 0: gradient step; mode 1: write A and B only (no update)
hipError_t run_attract(pixelsne_ctx* c, double alpha, void* A, void* B);
hipError_t run_finalize(pixelsne_ctx* c, int advance);
// the passes of one iteration without the renumbering
hipError_t run_iteration_passes(pixelsne_ctx* c);
// one iteration with events recorded before each pass and after the last (9 events)
hipError_t run_iteration_timed(pixelsne_ctx* c, hipEvent_t* ev);
hipError_t run_init_state(pixelsne_ctx* c, const double* Y, uint64_t seed, double sigma);
hipError_t run_get_y(const pixelsne_ctx* c, void* out, int frame);
hipError_t run_set_state(pixelsne_ctx* c, const void* z, const void* u, const void* g);
hipError_t run_get_state(const pixelsne_ctx* c, void* z, void* u, void* g);
hipError_t run_export_tree(const pixelsne_ctx* c, uint32_t* keys, uint32_t* perm,
                           uint32_t* prefix, uint32_t* count, double* sum);
hipError_t run_convert_val(pixelsne_ctx* c, const double* val64);
// exact-Z KL of the current state (synchronises); partial sums in a
// hipMalloc'd buffer, or (run_kl_static) in the library's fixed per-device
// array of kKlScratchDoubles doubles, for n up to kKlStaticMaxN
hipError_t run_kl(const pixelsne_ctx* c, double* kl);
hipError_t run_kl_static(const pixelsne_ctx* c, double* kl);
constexpr int64_t kKlStaticMaxN = (int64_t)1 << 24;
constexpr int64_t kKlScratchDoubles = kKlStaticMaxN / 256 + 2 * 4096 + 3;
int64_t kl_scratch_doubles(int64_t n);
// device address of the fixed KL array on `device` (which must be current the
// first time; resolved once per device)
hipError_t kl_scratch_address(int device, double** out);
// renumbering and the chunked copy of P (reorder.hip)
hipError_t run_reorder(pixelsne_ctx* c);
hipError_t run_scheduled_reorder(pixelsne_ctx* c);
// put the renumbering schedule where it stands after t iterations from the start
void reset_reorder_schedule(pixelsne_ctx* c, int32_t t);
hipError_t run_identity_order(pixelsne_ctx* c);
// renumber by a Morton code of three random projections of X (rows of D
// elements of x_dtype) and delay the first renumbering by the embedding to the
// end of the early exaggeration
hipError_t run_data_order(pixelsne_ctx* c, const void* X, int32_t D, int32_t x_dtype);
// P in the caller's numbering; row_ptr/col/val device, caller-owned
hipError_t run_export_P(const pixelsne_ctx* c, int64_t* row_ptr, int32_t* col, double* val);
// checks a caller's CSR (offsets monotone from 0 to nnz, columns in range and
// off the diagonal); *bad (host) = number of violations.  Synchronises.
hipError_t run_check_csr(const pixelsne_ctx* c, int64_t* bad);
hipError_t check_csr(const int64_t* row_ptr, const uint32_t* col, int64_t n, int64_t nnz,
                     hipStream_t s, int64_t* bad);
// scatter an internal-order [n][2] state-type array to caller order
hipError_t run_to_user_v2(const pixelsne_ctx* c, const void* in, void* out);
hipError_t run_map_perm(const pixelsne_ctx* c, const uint32_t* perm, uint32_t* out);
hipError_t scan_i64(const int64_t* a, int64_t m, int64_t* out, int64_t* tmp, hipStream_t s);
int64_t scan_i64_tmp_len(int64_t m);

// setup passes (setup.hip)
// 30-bit Morton code of three random (+-1) projections of each row of X,
// each quantised to 10 bits over its range; keys device uint32 [n]
hipError_t projection_keys(const void* X, int64_t n, int32_t D, int32_t x_dtype, uint32_t* keys,
                           hipStream_t s);
hipError_t knn(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k, int32_t* idx,
               double* d2, hipStream_t s, std::string* err);
// approximate kNN (knn_approx.hip): random-projection trees and rounds of
// neighbour exploring; leaf >= 2k + 2; same outputs as knn
hipError_t knn_approx(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k,
                      int32_t trees, int32_t leaf, int32_t explore, uint64_t seed, int32_t* idx,
                      double* d2, hipStream_t s, std::string* err);
hipError_t perplexity(const double* d2, int64_t n, int32_t k, double u, double* P,
                      double* beta, hipStream_t s);
// Symmetric CSR from kNN + conditional P.  Allocates row_ptr/col/val64 with
// hipMalloc (caller frees); synchronises once to read nnz.
hipError_t symmetrize(const int32_t* idx, const double* Pc, int64_t n, int32_t k,
                      int64_t** row_ptr, uint32_t** col, double** val64, int64_t* nnz,
                      hipStream_t s);

}  // namespace psne
