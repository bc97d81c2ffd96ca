// C ABI of the gfx950 PixelSNE library (declared in include/pixelsne.h).
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "ctx.h"

namespace psne {

int64_t attract_block_count(int64_t n);

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }

psne_status device_error(pixelsne_ctx* c, hipError_t e, const char* where) {
    if (c) c->poisoned = true;
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PSNE_E_NOMEM : PSNE_E_DEVICE;
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

namespace {

psne_status invalid(const std::string& m) {
    set_error(m);
    return PSNE_E_INVAL;
}

int log2_pow2(int32_t r) {
    if (r < 2 || (r & (r - 1))) return -1;
    int L = 0;
    while ((1 << L) < r) L++;
    return L;
}

psne_status check_params(const pixelsne_params* p) {
    if (p->struct_size != sizeof(pixelsne_params))
        return invalid("pixelsne_params.struct_size does not match this library");
    if (!(p->theta >= 0.0 && p->theta <= 0.99)) return invalid("theta must be in [0, 0.99]");
    if (!(p->eta > 0.0) || !(p->exaggeration > 0.0)) return invalid("eta and exaggeration must be > 0");
    if (!(p->min_gain >= 0.0) || !(p->eps > 0.0)) return invalid("min_gain >= 0 and eps > 0 required");
    if (p->precision != PSNE_FP32 && p->precision != PSNE_FP64) return invalid("unknown precision");
    if (p->com_mode != PSNE_COM_MASS && p->com_mode != PSNE_COM_CELL_CENTER)
        return invalid("unknown com_mode");
    if (p->x_dtype != PSNE_X_F32 && p->x_dtype != PSNE_X_F64 && p->x_dtype != PSNE_X_U8)
        return invalid("unknown x_dtype");
    if (p->exag_iters < 0 || p->mom_switch < 0) return invalid("negative schedule length");
    if (p->reorder_every < 0) return invalid("reorder_every must be >= 0");
    if (!(p->reorder_growth >= 1.0 && p->reorder_growth <= 1e6))
        return invalid("reorder_growth must be in [1, 1e6]");
    if (p->graphs != 0 && p->graphs != 1) return invalid("graphs must be 0 or 1");
    if (p->data_order != 0 && p->data_order != 1) return invalid("data_order must be 0 or 1");
    if (p->opening_fp64 != 0 && p->opening_fp64 != 1) return invalid("opening_fp64 must be 0 or 1");
    if (p->tree != PSNE_TREE_PIXEL && p->tree != PSNE_TREE_DATA) return invalid("unknown tree");
    if (p->knn_trees < 0 || p->knn_leaf < 0 || p->knn_explore < 0)
        return invalid("knn_trees, knn_leaf and knn_explore must be >= 0");
    if (p->attract_blocks_per_cu < 0 || p->attract_blocks_per_cu > 16)
        return invalid("attract_blocks_per_cu must be in [0, 16]");
    if (p->attract_help_blocks_per_cu < 0 || p->attract_help_blocks_per_cu > 16)
        return invalid("attract_help_blocks_per_cu must be in [0, 16]");
    if (p->attract_blocks_per_cu == 0 && p->attract_help_blocks_per_cu == 0)
        return invalid("attract_blocks_per_cu and attract_help_blocks_per_cu are both 0");
    if (p->attract_fork != PSNE_FORK_SNAP && p->attract_fork != PSNE_FORK_CELLS &&
        p->attract_fork != PSNE_FORK_AUTO)
        return invalid("unknown attract_fork");
    if (p->tree == PSNE_TREE_DATA && p->com_mode != PSNE_COM_MASS) {
        set_error("the data-driven tree takes centres of mass only (PSNE_COM_MASS)");
        return PSNE_E_UNSUPPORTED;
    }
    return PSNE_OK;
}

psne_status check_screen(int32_t w, int32_t h, int* L) {
    if (w < 2 || h < 2 || w > 65536 || h > 65536) return invalid("screen size must be in [2, 65536]");
    if (w != h) {
        set_error("only square screens are supported");
        return PSNE_E_UNSUPPORTED;
    }
    *L = log2_pow2(w);
    if (*L < 0) {
        set_error("screen size must be a power of two");
        return PSNE_E_UNSUPPORTED;
    }
    return PSNE_OK;
}

template <typename P>
hipError_t dalloc(pixelsne_ctx* c, P** out, size_t bytes) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
    if (e != hipSuccess) return e;
    c->allocs.push_back(p);
    *out = (P*)p;
    return hipSuccess;
}

size_t state_bytes(const pixelsne_ctx* c) { return c->prm.precision == PSNE_FP64 ? 8 : 4; }

hipError_t alloc_iteration_buffers(pixelsne_ctx* c) {
    const int64_t n = c->n;
    const size_t v2 = (size_t)n * 2 * state_bytes(c);
    hipError_t e;
    if ((e = dalloc(c, &c->zh, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->z, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->u, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->g, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->R, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->A, v2)) != hipSuccess) return e;
    if ((e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&c->ev_cells, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess) return e;
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device)) !=
        hipSuccess)
        return e;
    c->side_blocks = (int64_t)c->prm.attract_blocks_per_cu * (cus > 0 ? cus : 1);
    c->help_blocks = (int64_t)c->prm.attract_help_blocks_per_cu * (cus > 0 ? cus : 1);
    c->zpart_n = ceil_div(n, 256);
    if ((e = dalloc(c, &c->zpart, sizeof(double) * c->zpart_n)) != hipSuccess) return e;
    c->mm_n = attract_block_count(n);
    if ((e = dalloc(c, &c->mm_part, sizeof(double) * 4 * c->mm_n)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->sc, sizeof(DevScalars))) != hipSuccess) return e;
    TreeBufs& tb = c->tb;
    const bool dtree = c->prm.tree == PSNE_TREE_DATA;
    const int lmax = dtree ? kDLevels : c->L;       // deepest level of the tree
    int64_t mx = 0;
    for (int l = 0; l <= lmax; l++) {
        const int64_t cap = l < 31 ? (int64_t)1 << (2 * l) : n;
        mx += cap < n ? cap : n;
    }
    tb.max_nodes = mx;
    if (mx >= (int64_t)1 << 30) {
        set_error("too many tree cells: cell indices are limited to 2^30");
        return hipErrorNotSupported;
    }
    tb.sort_blocks = ceil_div(n, 2048);
    tb.tree_blocks = ceil_div(n, 256);
    for (int h = 0; h < 2; h++) {
        if ((e = dalloc(c, &tb.key[h], 4 * (size_t)n)) != hipSuccess) return e;
        if ((e = dalloc(c, &tb.idx[h], 4 * (size_t)n)) != hipSuccess) return e;
    }
    if ((e = dalloc(c, &tb.hist, 4 * 256 * (size_t)tb.sort_blocks)) != hipSuccess) return e;
    if ((e = dalloc(c, &tb.dtot, 4 * 256)) != hipSuccess) return e;
    if ((e = dalloc(c, &tb.lvl_cnt, 4 * (size_t)(lmax + 1) * tb.tree_blocks)) != hipSuccess) return e;
    if ((e = dalloc(c, &tb.ltot, 4 * (size_t)(lmax + 1))) != hipSuccess) return e;
    if (dtree) {
        for (int h = 0; h < 2; h++)
            if ((e = dalloc(c, &tb.key64[h], 8 * (size_t)n)) != hipSuccess) return e;
        if ((e = dalloc(c, &tb.cursor, 4 * (size_t)(mx + 1))) != hipSuccess) return e;
    }
    if ((e = dalloc(c, &tb.wfirst, sizeof(double2) * (size_t)ceil_div(n, 64))) != hipSuccess) return e;
    if ((e = dalloc(c, &tb.wlast, sizeof(double2) * (size_t)ceil_div(n, 64))) != hipSuccess) return e;
    if ((e = dalloc(c, &tb.first_child, 4 * (size_t)mx)) != hipSuccess) return e;
    if (!dtree && (e = dalloc(c, &tb.cell_start, 4 * (size_t)mx)) != hipSuccess) return e;
    // + 3: the traversal loads a sibling group as four records at once
    if ((e = dalloc(c, &tb.nodes, sizeof(Node) * (size_t)(mx + 3))) != hipSuccess) return e;
    if ((e = dalloc(c, &tb.nsum, sizeof(double2) * (size_t)mx)) != hipSuccess) return e;
    if (c->prm.precision == PSNE_FP32 && !c->prm.opening_fp64 &&
        (e = dalloc(c, &tb.cells32, sizeof(CellF) * (size_t)(mx + 3))) != hipSuccess)
        return e;
    if ((e = dalloc(c, &tb.leaf_of, 4 * (size_t)n)) != hipSuccess) return e;
    if ((e = dalloc(c, &tb.zs, v2)) != hipSuccess) return e;
    // renumbering: spare copies of the state, index maps, the chunked copy of P
    if ((e = dalloc(c, &c->orig, 4 * (size_t)n)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->orig2, 4 * (size_t)n)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->inv, 4 * (size_t)n)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->rp_int, 8 * (size_t)(n + 1))) != hipSuccess) return e;
    if ((e = dalloc(c, &c->ch_row, 4 * (size_t)(n + 1))) != hipSuccess) return e;
    if ((e = dalloc(c, &c->ch_tmp, 8 * (size_t)(n + 1))) != hipSuccess) return e;
    // FP32: column words and values interleaved in pk; FP64: values in vch
    if (c->prm.precision == PSNE_FP64) {
        if ((e = dalloc(c, &c->pk, 4 * (size_t)c->nnz)) != hipSuccess) return e;
        if ((e = dalloc(c, &c->vch, 8 * (size_t)c->nnz)) != hipSuccess) return e;
    } else {
        if ((e = dalloc(c, &c->pk, 8 * (size_t)c->nnz)) != hipSuccess) return e;
    }
    if ((e = dalloc(c, &c->zh2, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->u2, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->g2, v2)) != hipSuccess) return e;
    if ((e = dalloc(c, &c->len_tmp, 8 * (size_t)(n + 1))) != hipSuccess) return e;
    if ((e = dalloc(c, &c->scan_tmp, 8 * (size_t)scan_i64_tmp_len(n + 1))) != hipSuccess) return e;
    return hipSuccess;
}

void free_ctx(pixelsne_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    // the second stream's work is joined into the context's stream, except
    // after an error between the fork and the join
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (hipGraphExec_t& g : c->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_cells) (void)hipEventDestroy(c->ev_cells);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (void* p : c->allocs) (void)hipFree(p);
    delete c;
}

// The iteration's passes captured once per state-buffer parity on a private
// stream (nothing runs during the capture) and replayed on the caller's stream.
hipError_t capture_iteration(pixelsne_ctx* c, hipGraphExec_t* out) {
    hipError_t e = hipSuccess;
    if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    hipError_t e1 = e == hipSuccess ? run_iteration_passes(c) : e;
    hipGraph_t g = nullptr;
    if (e == hipSuccess) e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    if (e == hipSuccess) e = e1;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

hipError_t step_one(pixelsne_ctx* c) {
    hipError_t e = hipSuccess;
    bool done = false;
    if (c->prm.graphs && !c->graph_failed) {
        hipGraphExec_t& ge = c->gexec[c->parity];
        if (!ge && capture_iteration(c, &ge) != hipSuccess) {
            // capture unavailable: launch the kernels directly from now on
            (void)hipGetLastError();
            if (ge) (void)hipGraphExecDestroy(ge);
            ge = nullptr;
            c->graph_failed = true;
        }
        if (ge) {
            e = hipGraphLaunch(ge, c->stream);
            done = true;
        }
    }
    if (!done) e = run_iteration_passes(c);
    if (e == hipSuccess) e = run_scheduled_reorder(c);
    return e;
}

pixelsne_ctx* new_ctx(int64_t n, int L, int32_t r, const pixelsne_params* p) {
    pixelsne_ctx* c = new pixelsne_ctx();
    c->n = n;
    c->L = L;
    c->r = r;
    c->prm = *p;
    c->stream = (hipStream_t)p->stream;
    (void)hipGetDevice(&c->device);
    return c;
}

// state buffers + initial embedding; P must already be in the context
psne_status finish_init(pixelsne_ctx* c) {
    hipError_t e = alloc_iteration_buffers(c);
    if (e == hipErrorNotSupported) return PSNE_E_UNSUPPORTED;
    if (e != hipSuccess) return device_error(c, e, "allocation");
    if (c->prm.Y_init && !is_device_ptr(c->prm.Y_init)) return invalid("Y_init must be a device pointer");
    // the initial state resets the device scalars; the chunked P (whose chunk
    // count lives there) is built after it
    // the device address of the library's fixed KL array on this device
    // (pixelsne_kl_noalloc), resolved once per device while it is current
    double* kl_fixed = nullptr;
    e = kl_scratch_address(c->device, &kl_fixed);
    if (e != hipSuccess) return device_error(c, e, "resolving the fixed KL buffer");
    e = run_init_state(c, c->prm.Y_init, c->prm.seed, c->prm.init_sigma);
    if (e == hipSuccess) e = run_identity_order(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(c, e, "initial embedding");
    return PSNE_OK;
}

}  // namespace
}  // namespace psne

using namespace psne;

extern "C" {

const char* pixelsne_last_error(void) { return g_err.c_str(); }

void pixelsne_default_params(pixelsne_params* p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(pixelsne_params);
    p->k = 0;
    p->theta = 0.5;
    p->exag_iters = 250;
    p->exaggeration = 12.0;
    p->eta = 200.0;
    p->mom0 = 0.5;
    p->mom1 = 0.8;
    p->mom_switch = 250;
    p->min_gain = 0.01;
    p->eps = 1e-6;
    p->init_sigma = 1e-4;
    p->seed = 0;
    p->precision = PSNE_FP32;
    p->com_mode = PSNE_COM_MASS;
    p->x_dtype = PSNE_X_F32;
    p->Y_init = nullptr;
    p->stream = nullptr;
    p->reorder_every = 100;
    p->data_order = 1;
    p->graphs = 1;
    p->reorder_growth = 2.0;
    p->opening_fp64 = 0;
    p->tree = PSNE_TREE_PIXEL;
    p->knn_trees = 0;
    p->knn_leaf = 0;
    p->knn_explore = 1;
    p->attract_blocks_per_cu = 2;
    p->attract_help_blocks_per_cu = 3;
    p->attract_fork = PSNE_FORK_AUTO;
}

pixelsne_ctx* pixelsne_init_ex(const void* X, int64_t n, int32_t D, double perplexity,
                               int32_t screen_w, int32_t screen_h, const pixelsne_params* pin) {
    pixelsne_params p;
    if (pin) p = *pin;
    else pixelsne_default_params(&p);
    if (check_params(&p) != PSNE_OK) return nullptr;
    if (n < 2 || n >= ((int64_t)1 << kColBits)) { invalid("n must be in [2, 2^27)"); return nullptr; }
    if (D < 1) { invalid("D must be >= 1"); return nullptr; }
    if (!(perplexity > 0.0) || !isfinite(perplexity)) { invalid("perplexity must be > 0"); return nullptr; }
    const int64_t k = p.k > 0 ? p.k : (int64_t)floor(3.0 * perplexity);
    if (k < 1 || k > n - 1) { invalid("k = floor(3 * perplexity) must be in [1, n - 1]"); return nullptr; }
    if (k > 256) { set_error("k > 256 is not supported"); return nullptr; }
    int L;
    if (check_screen(screen_w, screen_h, &L) != PSNE_OK) return nullptr;
    if (!is_device_ptr(X)) { invalid("X must be a device pointer"); return nullptr; }

    pixelsne_ctx* c = new_ctx(n, L, screen_w, &p);
    c->k = (int32_t)k;
    int32_t* idx = nullptr;
    double *d2 = nullptr, *Pc = nullptr, *val64 = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(idx); (void)hipFree(d2); (void)hipFree(Pc); (void)hipFree(val64);
    };
    hipError_t e = hipMalloc(&idx, sizeof(int32_t) * n * k);
    if (e == hipSuccess) e = hipMalloc(&d2, sizeof(double) * n * k);
    if (e == hipSuccess) e = hipMalloc(&Pc, sizeof(double) * n * k);
    std::string err;
    const int32_t leaf = p.knn_leaf > 0 ? p.knn_leaf : (int32_t)(2 * k + 2);
    if (p.knn_trees > 0 && leaf < 2 * k + 2) {
        invalid("knn_leaf must be >= 2k + 2");
        cleanup();
        free_ctx(c);
        return nullptr;
    }
    if (e == hipSuccess)
        e = p.knn_trees > 0
                ? psne::knn_approx(X, n, D, p.x_dtype, (int32_t)k, p.knn_trees, leaf,
                                   p.knn_explore, p.seed, idx, d2, c->stream, &err)
                : psne::knn(X, n, D, p.x_dtype, (int32_t)k, idx, d2, c->stream, &err);
    if (e == hipSuccess) e = psne::perplexity(d2, n, (int32_t)k, perplexity, Pc, nullptr, c->stream);
    int64_t* rp = nullptr;
    uint32_t* col = nullptr;
    if (e == hipSuccess)
        e = psne::symmetrize(idx, Pc, n, (int32_t)k, &rp, &col, &val64, &c->nnz, c->stream);
    if (e != hipSuccess) {
        if (!err.empty()) set_error(err);
        else device_error(c, e, "building P");
        cleanup();
        free_ctx(c);
        return nullptr;
    }
    c->allocs.push_back(rp);
    c->allocs.push_back(col);
    c->row_ptr = rp;
    c->col = col;
    e = dalloc(c, &c->val, (size_t)c->nnz * state_bytes(c));
    if (e == hipSuccess) e = run_convert_val(c, val64);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    cleanup();
    if (e != hipSuccess) { device_error(c, e, "storing P"); free_ctx(c); return nullptr; }
    if (finish_init(c) != PSNE_OK) { free_ctx(c); return nullptr; }
    if (p.data_order) {
        e = run_data_order(c, X, D, p.x_dtype);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) { device_error(c, e, "data order"); free_ctx(c); return nullptr; }
    }
    return c;
}

pixelsne_ctx* pixelsne_init(const float* X, int64_t n, int32_t D, double perplexity,
                            int32_t screen_w, int32_t screen_h) {
    pixelsne_params p;
    pixelsne_default_params(&p);
    return pixelsne_init_ex(X, n, D, perplexity, screen_w, screen_h, &p);
}

pixelsne_ctx* pixelsne_init_with_P(int64_t n, int64_t nnz, const int64_t* row_ptr,
                                   const int32_t* col, const double* val, int32_t screen_w,
                                   int32_t screen_h, const pixelsne_params* pin) {
    pixelsne_params p;
    if (pin) p = *pin;
    else pixelsne_default_params(&p);
    if (check_params(&p) != PSNE_OK) return nullptr;
    if (n < 2 || n >= ((int64_t)1 << kColBits)) { invalid("n must be in [2, 2^27)"); return nullptr; }
    if (nnz < 1) { invalid("nnz must be >= 1"); return nullptr; }
    int L;
    if (check_screen(screen_w, screen_h, &L) != PSNE_OK) return nullptr;
    if (!is_device_ptr(row_ptr) || !is_device_ptr(col) || !is_device_ptr(val)) {
        invalid("row_ptr, col and val must be device pointers");
        return nullptr;
    }
    pixelsne_ctx* c = new_ctx(n, L, screen_w, &p);
    c->nnz = nnz;
    hipError_t e = dalloc(c, &c->row_ptr, 8 * (size_t)(n + 1));
    if (e == hipSuccess) e = dalloc(c, &c->col, 4 * (size_t)nnz);
    if (e == hipSuccess) e = dalloc(c, &c->val, state_bytes(c) * (size_t)nnz);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->row_ptr, row_ptr, 8 * (size_t)(n + 1), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->col, col, 4 * (size_t)nnz, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = run_convert_val(c, val);
    int64_t bad = 0;
    if (e == hipSuccess) e = run_check_csr(c, &bad);
    if (e != hipSuccess) { device_error(c, e, "copying P"); free_ctx(c); return nullptr; }
    if (bad) {
        invalid("P is not a valid CSR (row_ptr from 0 to nnz, ascending; columns in [0, n) and off "
                "the diagonal)");
        free_ctx(c);
        return nullptr;
    }
    if (finish_init(c) != PSNE_OK) { free_ctx(c); return nullptr; }
    return c;
}

psne_status pixelsne_step_async(pixelsne_ctx* c, int32_t n_iter) {
    if (!c) return invalid("null context");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    if (n_iter < 0) return invalid("n_iter must be >= 0");
    for (int32_t it = 0; it < n_iter; it++) {
        hipError_t e = step_one(c);
        if (e != hipSuccess) return device_error(c, e, "iteration");
    }
    return PSNE_OK;
}

psne_status pixelsne_step(pixelsne_ctx* c, int32_t n_iter) {
    psne_status st = pixelsne_step_async(c, n_iter);
    if (st != PSNE_OK) return st;
    int32_t bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, &c->sc->nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(c, e, "step");
    if (bad) {
        set_error("non-finite positions");
        return PSNE_E_NUMERIC;
    }
    return PSNE_OK;
}

psne_status pixelsne_step_profiled(pixelsne_ctx* c, int32_t n_iter, pixelsne_pass_times* out) {
    if (!c || !out) return invalid("null argument");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    if (n_iter < 0) return invalid("n_iter must be >= 0");
    memset(out, 0, sizeof(*out));
    constexpr int kEv = 13;     // pass boundaries of one iteration (see run_iteration_timed)
    std::vector<hipEvent_t> ev((size_t)n_iter * kEv);
    hipError_t e = hipSuccess;
    size_t made = 0;
    for (; made < ev.size() && e == hipSuccess; made++) e = hipEventCreate(&ev[made]);
    if (e != hipSuccess) made--;
    for (int32_t it = 0; it < n_iter && e == hipSuccess; it++)
        e = run_iteration_timed(c, &ev[(size_t)kEv * it]);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    double* acc[8] = {&out->snap_ms, &out->sort_ms, &out->tree_ms, &out->traverse_ms,
                      &out->zsum_ms, &out->attract_ms, &out->finalize_ms, &out->reorder_ms};
    // (from, to) events of each pass: main-stream passes, the row sums on
    // the second stream (its two launches: one of them leaves at once),
    // update + scaling from the join, renumbering
    const int span[9][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {9, 10}, {6, 7}, {7, 8},
                            {11, 12}};
    const int into[9] = {0, 1, 2, 3, 4, 5, 6, 7, 5};
    for (int32_t it = 0; it < n_iter && e == hipSuccess; it++)
        for (int p = 0; p < 9 && e == hipSuccess; p++) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[(size_t)kEv * it + span[p][0]],
                                    ev[(size_t)kEv * it + span[p][1]]);
            *acc[into[p]] += ms;
        }
    for (size_t i = 0; i < made; i++) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return device_error(c, e, "step_profiled");
    out->iterations = n_iter;
    int32_t bad = 0;
    e = hipMemcpy(&bad, &c->sc->nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_error(c, e, "step_profiled");
    if (bad) { set_error("non-finite positions"); return PSNE_E_NUMERIC; }
    return PSNE_OK;
}

psne_status pixelsne_get_Y(const pixelsne_ctx* c, void* out, int32_t frame) {
    if (!c) return invalid("null context");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    if (frame != PSNE_FRAME_PIXEL && frame != PSNE_FRAME_SCREEN && frame != PSNE_FRAME_Y)
        return invalid("unknown frame");
    if (!is_device_ptr(out)) return invalid("out must be a device pointer");
    hipError_t e = run_get_y(c, out, frame);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "get_Y");
    return PSNE_OK;
}

void pixelsne_destroy(pixelsne_ctx* c) { free_ctx(c); }

psne_status pixelsne_get_stats(const pixelsne_ctx* c, pixelsne_stats* out) {
    if (!c || !out) return invalid("null argument");
    DevScalars h;
    hipError_t e = hipMemcpyAsync(&h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "get_stats");
    memset(out, 0, sizeof(*out));
    out->n = c->n;
    out->nnz = c->nnz;
    out->n_nodes = h.n_nodes;
    out->r = c->r;
    out->L = c->L;
    out->k = c->k;
    out->precision = c->prm.precision;
    out->com_mode = c->prm.com_mode;
    out->iteration = h.t;
    out->s[0] = h.s[0];
    out->s[1] = h.s[1];
    out->Z = h.Z;
    for (int l = 0; l <= c->L && l < 17; l++) out->level_size[l] = h.level_size[l];
    out->renumberings = c->scheduled_reorders;
    out->fork_cells = h.fork_late;
    int khz = 0;   // the device wall clock's rate
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "get_stats");
    if (khz > 0)
        for (int k = 0; k < 2; k++) out->fork_ms[k] = (double)h.fork_ticks[k] / (double)khz;
    return PSNE_OK;
}

psne_status pixelsne_set_state(pixelsne_ctx* c, const void* z, const void* u, const void* g,
                               const double* s, int32_t iteration) {
    if (!c) return invalid("null context");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    if (!is_device_ptr(z) || (u && !is_device_ptr(u)) || (g && !is_device_ptr(g)))
        return invalid("z, u, g must be device pointers");
    if (!s || !(s[0] > 0.0) || !(s[1] > 0.0)) return invalid("s must hold two positive scales");
    if (iteration < 0) return invalid("iteration must be >= 0");
    DevScalars h;
    hipError_t e = hipMemcpyAsync(&h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(c, e, "set_state");
    h.s[0] = s[0];
    h.s[1] = s[1];
    h.zmin[0] = h.zmin[1] = 0.0;
    h.scale[0] = h.scale[1] = 1.0;
    h.uscale[0] = h.uscale[1] = 1.0;
    h.t = iteration;
    h.nonfinite = 0;
    reset_fork_tuner(h, c->prm.attract_fork);
    e = hipMemcpyAsync(c->sc, &h, sizeof(h), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = run_set_state(c, z, u, g);
    // the renumbering schedule as it stands after `iteration` iterations (the
    // points keep their current internal numbering)
    reset_reorder_schedule(c, iteration);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(c, e, "set_state");
    return PSNE_OK;
}

psne_status pixelsne_get_state(const pixelsne_ctx* c, void* z, void* u, void* g, double* s,
                               int32_t* iteration) {
    if (!c) return invalid("null context");
    if ((z && !is_device_ptr(z)) || (u && !is_device_ptr(u)) || (g && !is_device_ptr(g)))
        return invalid("z, u, g must be device pointers");
    hipError_t e = run_get_state(c, z, u, g);
    DevScalars h;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "get_state");
    if (s) { s[0] = h.s[0]; s[1] = h.s[1]; }
    if (iteration) *iteration = h.t;
    return PSNE_OK;
}

psne_status pixelsne_gradient(pixelsne_ctx* c, double alpha, void* B, void* A, void* R,
                              double* Zi, uint32_t* visits, uint32_t* used, double* Z) {
    if (!c) return invalid("null context");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    const void* ptrs[6] = {B, A, R, Zi, visits, used};
    for (const void* p : ptrs)
        if (p && !is_device_ptr(p)) return invalid("outputs must be device pointers");
    if (!isfinite(alpha)) return invalid("alpha must be finite");
    hipError_t e = run_snap(c);
    if (e == hipSuccess) e = run_sort(c);
    if (e == hipSuccess) e = run_tree(c);
    if (e == hipSuccess) e = run_traverse(c, visits, used, Zi);
    if (e == hipSuccess) e = run_zsum(c);
    if (e == hipSuccess) e = run_attract(c, alpha, A, B);
    if (e == hipSuccess && R) e = run_to_user_v2(c, c->R, R);
    double hz = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hz, &c->sc->Z, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(c, e, "gradient");
    if (Z) *Z = hz;
    return PSNE_OK;
}

psne_status pixelsne_export_tree(const pixelsne_ctx* c, int64_t* level_size, uint32_t* keys,
                                 uint32_t* perm, uint32_t* prefix, uint32_t* count, double* sum) {
    if (!c || !level_size) return invalid("null argument");
    if (c->prm.tree != PSNE_TREE_PIXEL) return invalid("pixelsne_export_tree64 exports the data-driven tree");
    const void* ptrs[5] = {keys, perm, prefix, count, sum};
    for (const void* p : ptrs)
        if (p && !is_device_ptr(p)) return invalid("outputs must be device pointers");
    DevScalars h;
    hipError_t e = hipMemcpyAsync(&h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "export_tree");
    for (int l = 0; l <= c->L; l++) level_size[l] = h.level_size[l];
    e = run_export_tree(c, keys, perm, prefix, count, sum);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "export_tree");
    return PSNE_OK;
}

psne_status pixelsne_export_tree64(const pixelsne_ctx* c, int64_t* level_size, uint64_t* keys,
                                   uint32_t* perm, uint64_t* prefix, uint32_t* count,
                                   double* sum) {
    if (!c || !level_size) return invalid("null argument");
    if (c->prm.tree != PSNE_TREE_DATA) return invalid("the context does not build the data-driven tree");
    const void* ptrs[5] = {keys, perm, prefix, count, sum};
    for (const void* p : ptrs)
        if (p && !is_device_ptr(p)) return invalid("outputs must be device pointers");
    DevScalars h;
    hipError_t e = hipMemcpyAsync(&h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "export_tree64");
    for (int l = 0; l <= kDLevels; l++) level_size[l] = h.level_size[l];
    e = run_export_dtree(c, keys, perm, prefix, count, sum);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "export_tree64");
    return PSNE_OK;
}

psne_status pixelsne_export_P(const pixelsne_ctx* c, int64_t* nnz, int64_t* row_ptr, int32_t* col,
                              double* val) {
    if (!c || !nnz) return invalid("null argument");
    *nnz = c->nnz;
    const void* ptrs[3] = {row_ptr, col, val};
    for (const void* p : ptrs)
        if (p && !is_device_ptr(p)) return invalid("outputs must be device pointers");
    hipError_t e = hipSuccess;
    if (row_ptr || col || val) e = run_export_P(c, row_ptr, col, val);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "export_P");
    return PSNE_OK;
}

psne_status pixelsne_kl(const pixelsne_ctx* c, double* kl) {
    if (!c || !kl) return invalid("null argument");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    hipError_t e = run_kl(c, kl);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "kl");
    return PSNE_OK;
}

psne_status pixelsne_kl_noalloc(const pixelsne_ctx* c, double* kl) {
    if (!c || !kl) return invalid("null argument");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    if (kl_scratch_doubles(c->n) > kKlScratchDoubles) {
        set_error("pixelsne_kl_noalloc supports n <= 2^24 (its fixed buffer holds " +
                  std::to_string(kKlScratchDoubles) + " partial sums); use pixelsne_kl");
        return PSNE_E_UNSUPPORTED;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != c->device) return invalid("the context's device must be current");
    if (e == hipSuccess) e = run_kl_static(c, kl);
    if (e != hipSuccess) return device_error(const_cast<pixelsne_ctx*>(c), e, "kl_noalloc");
    return PSNE_OK;
}

psne_status pixelsne_refine(pixelsne_ctx* c, double kl_target, int32_t check_every,
                            int32_t refine_iters, int32_t max_iters,
                            pixelsne_refine_result* out) {
    if (!c || !out) return invalid("null argument");
    if (c->poisoned) { set_error("context unusable after a device error"); return PSNE_E_STATE; }
    if (!isfinite(kl_target)) return invalid("kl_target must be finite");
    if (check_every < 1) return invalid("check_every must be >= 1");
    if (refine_iters < 0 || max_iters < refine_iters)
        return invalid("0 <= refine_iters <= max_iters required");
    memset(out, 0, sizeof(*out));
    hipError_t e = run_kl(c, &out->kl_start);
    if (e != hipSuccess) return device_error(c, e, "refine");
    out->kl = out->kl_start;
    out->reached = out->kl <= kl_target ? 1 : 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    int32_t done = 0;
    double ms_total = 0.0;
    psne_status st = PSNE_OK;
    while (e == hipSuccess && !out->reached && done < max_iters) {
        const int32_t chunk = check_every < max_iters - done ? check_every : max_iters - done;
        e = hipEventRecord(ev[0], c->stream);
        if (e != hipSuccess) break;
        st = pixelsne_step_async(c, chunk);
        if (st != PSNE_OK) break;
        e = hipEventRecord(ev[1], c->stream);
        int32_t bad = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&bad, &c->sc->nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost,
                               c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) break;
        ms_total += ms;
        done += chunk;
        if (bad) {
            set_error("non-finite positions");
            st = PSNE_E_NUMERIC;
            break;
        }
        e = run_kl(c, &out->kl);
        out->reached = e == hipSuccess && out->kl <= kl_target ? 1 : 0;
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    out->iterations = done;
    out->iter_ms = ms_total;
    // the refinement budget did not reach the target: the iterations past it
    // (or all of max_iters) were the plain method's
    out->fallback = (done > refine_iters || !out->reached) ? 1 : 0;
    if (e != hipSuccess) return device_error(c, e, "refine");
    return st;
}

psne_status pixelsne_knn(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k,
                         int32_t* idx, double* d2, void* stream) {
    if (n < 2 || n >= ((int64_t)1 << 31)) return invalid("n must be in [2, 2^31)");
    if (D < 1) return invalid("D must be >= 1");
    if (k < 1 || k > n - 1 || k > 256) return invalid("k must be in [1, min(n - 1, 256)]");
    if (x_dtype != PSNE_X_F32 && x_dtype != PSNE_X_F64 && x_dtype != PSNE_X_U8)
        return invalid("unknown x_dtype");
    if (!is_device_ptr(X) || !is_device_ptr(idx) || !is_device_ptr(d2))
        return invalid("X, idx, d2 must be device pointers");
    std::string err;
    hipError_t e = psne::knn(X, n, D, x_dtype, k, idx, d2, (hipStream_t)stream, &err);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess && !err.empty()) {
        set_error(err);
        return PSNE_E_NUMERIC;
    }
    if (e != hipSuccess) return device_error(nullptr, e, "knn");
    return PSNE_OK;
}

psne_status pixelsne_knn_approx(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k,
                                int32_t trees, int32_t leaf_size, int32_t explore,
                                uint64_t seed, int32_t* idx, double* d2, void* stream) {
    if (n < 2 || n >= ((int64_t)1 << 31)) return invalid("n must be in [2, 2^31)");
    if (D < 1) return invalid("D must be >= 1");
    if (k < 1 || k > n - 1 || k > 256) return invalid("k must be in [1, min(n - 1, 256)]");
    if (trees < 1 || explore < 0) return invalid("trees >= 1 and explore >= 0 required");
    const int32_t leaf = leaf_size > 0 ? leaf_size : 2 * k + 2;
    if (leaf < 2 * k + 2) return invalid("leaf_size must be >= 2k + 2");
    if (x_dtype != PSNE_X_F32 && x_dtype != PSNE_X_F64 && x_dtype != PSNE_X_U8)
        return invalid("unknown x_dtype");
    if (!is_device_ptr(X) || !is_device_ptr(idx) || !is_device_ptr(d2))
        return invalid("X, idx, d2 must be device pointers");
    std::string err;
    hipError_t e = psne::knn_approx(X, n, D, x_dtype, k, trees, leaf, explore, seed, idx, d2,
                                    (hipStream_t)stream, &err);
    if (e != hipSuccess && !err.empty()) {
        set_error(err);
        return PSNE_E_DEVICE;
    }
    if (e != hipSuccess) return device_error(nullptr, e, "knn_approx");
    return PSNE_OK;
}

psne_status pixelsne_perplexity(const double* d2, int64_t n, int32_t k, double perplexity,
                                double* P, double* beta, void* stream) {
    if (n < 1 || k < 1) return invalid("n and k must be >= 1");
    if (!(perplexity > 0.0)) return invalid("perplexity must be > 0");
    if (!is_device_ptr(d2) || !is_device_ptr(P) || (beta && !is_device_ptr(beta)))
        return invalid("d2, P, beta must be device pointers");
    hipError_t e = psne::perplexity(d2, n, k, perplexity, P, beta, (hipStream_t)stream);
    if (e != hipSuccess) return device_error(nullptr, e, "perplexity");
    return PSNE_OK;
}

}  // extern "C"
