// batch.cpp -- uneven-size batches: many sinograms of different sizes in one
// graph launch (the paper processes blocks of Q sinograms at once, Section 2;
// its pipeline tunes block sizes and queue lengths per stage, Section 3).
//
// Instances are grouped into classes of equal (n, V); each class gets its own
// plan (tables for its angle count) and its own workspace region, so classes
// can run concurrently. Kernels read the instances' sinograms and write their
// images through per-slice pointer lists, so instances need not be contiguous
// or ordered by class. The first call with a given workspace captures every
// class's three launches into one hipGraph, forked over a few streams (all at
// default priority) and joined back; later calls update the pointer lists and
// replay the graph. bst_batch_tune times the gather kernel's variants per
// class on the caller's data and keeps the fastest before the capture.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "bst_internal.h"

namespace {

struct Class {
    int n, V;
    bst_plan_t plan = nullptr;
    std::vector<int> members;  // instance indices, in input order
    int list_base = 0;         // offset of this class's pointers in the lists
    size_t ws_off = 0, ws_bytes = 0;
};

constexpr int kStreams = 4;

}  // namespace

struct bst_batch_s {
    int device = 0;
    int count = 0;
    std::vector<Class> classes;
    size_t ws_total = 0;
    void* d_lists = nullptr;              // device: [count] sinogram then [count] image pointers
    const float** d_sino_list = nullptr;
    float** d_img_list = nullptr;
    void* h_lists = nullptr;              // pinned host staging, 2 * count pointers
    hipEvent_t lists_done = nullptr;      // the staging may be rewritten after this
    hipStream_t streams[kStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t joins[kStreams] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* graph_ws = nullptr;             // workspace the graph was captured with
};

namespace {

bst_status fail(hipError_t e) {
    bst::set_last_error(e);
    return BST_E_DEVICE;
}

void release(bst_batch_s* b) {
    if (!b) return;
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && prev != b->device) (void)hipSetDevice(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& c : b->classes)
        if (c.plan) (void)bst_destroy(c.plan);
    if (b->d_lists) (void)hipFree(b->d_lists);
    if (b->h_lists) (void)hipHostFree(b->h_lists);
    if (b->lists_done) (void)hipEventDestroy(b->lists_done);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (int i = 0; i < kStreams; ++i) {
        if (b->joins[i]) (void)hipEventDestroy(b->joins[i]);
        if (b->streams[i]) (void)hipStreamDestroy(b->streams[i]);
    }
    if (prev >= 0 && prev != b->device) (void)hipSetDevice(prev);
    delete b;
}

// Enqueue one class's spectrum, gather and row kernels on `st`.
hipError_t launch_class(const bst_batch_s* b, const Class& c, void* ws, hipStream_t st) {
    const bst_plan_s& p = *c.plan;
    const int batch = (int)c.members.size();
    bst::TentSizes tent;
    if (p.tent) {
        tent.W = p.tent_w;
        tent.rowsV = (size_t)p.tent_rows * (size_t)p.V;
        tent.C = p.tent_chunks;
    }
    const bst::WsLayout L = bst::workspace_layout(p.n, p.V, p.N, p.M, p.G, batch, p.prm.interp, p.monopole, tent);
    unsigned char* w = static_cast<unsigned char*>(ws) + c.ws_off;
    float2* polar = reinterpret_cast<float2*>(w + L.polar_off);
    float* dc = reinterpret_cast<float*>(w + L.dc_off);
    float2* grid = reinterpret_cast<float2*>(w + L.grid_off);
    float* mass = p.monopole ? reinterpret_cast<float*>(w + L.mass_off) : nullptr;
    hipError_t e;
    if (p.monopole) {
        const bst::MassArgs ma{nullptr, b->d_sino_list + c.list_base, nullptr, nullptr, mass, p.n, p.V};
        e = bst::launch_mass(p, ma, batch, st);
        if (e != hipSuccess) return e;
    }
    bst::SpecArgs sa{nullptr, b->d_sino_list + c.list_base, nullptr, nullptr, polar, dc, p.taper, p.kc,
                     p.tw_M, p.n, p.V, p.S, p.lead, p.S - p.lead - p.M / 2, (float)p.dt,
                     mass, p.mono_phi, p.mono_inv};
    e = bst::launch_spectrum(p, sa, batch, st);
    if (e != hipSuccess) return e;
    bst::GatherArgs ga{};
    ga.polar = polar;
    ga.dc = dc;
    ga.grid = grid;
    ga.tw = p.tw_G;
    ga.V = p.V;
    ga.S = p.S;
    ga.GT = p.GT;
    ga.N = p.N;
    ga.Mh = p.M / 2;
    ga.zero_slot = p.M / 2 + p.lead;
    ga.inv_gap = p.inv_gap;
    ga.uniform = p.uniform ? 1 : 0;
    ga.batch = batch;
    ga.slices_per_block = p.gather_slices;
    ga.rscale = p.rscale;
    ga.vpi_f = (float)p.vpi;
    ga.ang = p.ang;
    ga.dc_scale = p.dc_scale;
    if (p.tent) {
        float2* patch = reinterpret_cast<float2*>(w + L.tent_off);
        float2* trans = reinterpret_cast<float2*>(w + L.tent_trans_off);
        float2* part = reinterpret_cast<float2*>(w + L.tent_part_off);
        float* wsum = reinterpret_cast<float*>(w + L.tent_wsum_off);
        const bst::TentArgs ta{polar, trans, patch, part, wsum, p.tent_cols, p.tent_chunk, p.tent_coff,
                               (int)p.tent_w, (int)p.tent_chunks, p.V, p.S, p.lead, p.tent_rows, p.G / 2, p.rscale};
        e = bst::launch_tent(p, ta, batch, st);
        if (e != hipSuccess) return e;
        ga.tent_cols = p.tent_cols;
        ga.patch = patch;
        ga.tent_w = (int)p.tent_w;
    }
    e = bst::launch_gather_colifft(p, ga, st);
    if (e != hipSuccess) return e;
    bst::RowArgs ra{grid, nullptr, b->d_img_list + c.list_base, p.tw_G, p.N, p.GT, p.out_scale, 0,
                    mass, p.mono_inv, p.mono_amp, p.mono_rho_px};
    return bst::launch_row_c2r(p, ra, batch, st);
}

struct Guard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit Guard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~Guard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

bst_status bst_batch_create(const bst_params* base, int32_t count, const int32_t* n_det, const int32_t* n_angles,
                            bst_batch_t* out) {
    if (!out) return BST_E_NULL;
    *out = nullptr;
    if (!base || !n_det || !n_angles) return BST_E_NULL;
    if (count < 1) return BST_E_BATCH;
    if (base->angles) return BST_E_UNSUPPORTED;  // uniform angles only: V differs per instance
    if (base->dtype != BST_F32) return BST_E_UNSUPPORTED;
    std::map<std::pair<int, int>, int> index;
    std::vector<std::pair<int, int>> keys;
    std::vector<std::vector<int>> members;
    for (int i = 0; i < count; ++i) {
        bst_params p = *base;
        p.n_det = n_det[i];
        p.n_out = n_det[i];
        p.n_angles = n_angles[i];
        p.max_batch = 1;
        const bst_status st = bst_validate(&p);
        if (st != BST_OK) return st;
        const auto key = std::make_pair(n_det[i], n_angles[i]);
        auto it = index.find(key);
        if (it == index.end()) {
            index.emplace(key, (int)keys.size());
            keys.push_back(key);
            members.emplace_back();
            it = index.find(key);
        }
        members[it->second].push_back(i);
    }
    bst_batch_s* b = new (std::nothrow) bst_batch_s();
    if (!b) return BST_E_NOMEM;
    b->device = base->device;
    b->count = count;
    Guard guard(b->device);
    if (guard.err != hipSuccess) {
        delete b;
        return fail(guard.err);
    }
    int list_base = 0;
    size_t off = 0;
    for (size_t k = 0; k < keys.size(); ++k) {
        Class c;
        c.n = keys[k].first;
        c.V = keys[k].second;
        c.members = members[k];
        bst_params p = *base;
        p.n_det = c.n;
        p.n_out = c.n;
        p.n_angles = c.V;
        p.max_batch = (int32_t)c.members.size();
        p.adjoint = 0;
        const bst_status st = bst_plan(&p, &c.plan);
        if (st != BST_OK) {
            b->classes.push_back(c);
            release(b);
            return st;
        }
        c.list_base = list_base;
        list_base += (int)c.members.size();
        (void)bst_workspace_size(c.plan, p.max_batch, &c.ws_bytes);
        c.ws_off = off;
        off += (c.ws_bytes + 255) & ~(size_t)255;
        b->classes.push_back(c);
    }
    b->ws_total = off;
    hipError_t e = hipMalloc(&b->d_lists, 2 * (size_t)count * sizeof(void*));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_lists, 2 * (size_t)count * sizeof(void*), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->lists_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; e == hipSuccess && i < kStreams; ++i) {
        e = hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->joins[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release(b);
        return fail(e);
    }
    b->d_sino_list = static_cast<const float**>(b->d_lists);
    b->d_img_list = reinterpret_cast<float**>(static_cast<char*>(b->d_lists) + (size_t)count * sizeof(void*));
    *out = b;
    return BST_OK;
}

bst_status bst_batch_workspace_size(bst_batch_t b, size_t* bytes) {
    if (!b || !bytes) return BST_E_NULL;
    *bytes = b->ws_total;
    return BST_OK;
}

bst_status bst_batch_classes(bst_batch_t b, int32_t* n_classes) {
    if (!b || !n_classes) return BST_E_NULL;
    *n_classes = (int32_t)b->classes.size();
    return BST_OK;
}

// Host part shared by tune and run: check arguments and stage the pointer lists.
static bst_status stage_lists(bst_batch_t b, const float* sinos, const int64_t* sino_off, float* imgs,
                              const int64_t* img_off, void* ws, size_t ws_bytes, hipStream_t s) {
    if (!b || !sinos || !sino_off || !imgs || !img_off || !ws) return BST_E_NULL;
    if (ws_bytes < b->ws_total) return BST_E_WORKSPACE;
    hipError_t e = hipEventSynchronize(b->lists_done);  // previous upload has read the staging
    if (e != hipSuccess) return fail(e);
    const float** hs = static_cast<const float**>(b->h_lists);
    float** hi = reinterpret_cast<float**>(static_cast<char*>(b->h_lists) + (size_t)b->count * sizeof(void*));
    for (const auto& c : b->classes) {
        for (size_t k = 0; k < c.members.size(); ++k) {
            const int i = c.members[k];
            if (sino_off[i] < 0 || img_off[i] < 0) return BST_E_SHAPE;
            hs[c.list_base + k] = sinos + sino_off[i];
            hi[c.list_base + k] = imgs + img_off[i];
        }
    }
    e = hipMemcpyAsync(b->d_lists, b->h_lists, 2 * (size_t)b->count * sizeof(void*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(b->lists_done, s);
    return e == hipSuccess ? BST_OK : fail(e);
}

bst_status bst_batch_tune(bst_batch_t b, const float* sinos, const int64_t* sino_off, float* imgs,
                          const int64_t* img_off, void* ws, size_t ws_bytes, void* stream) {
    Guard guard(b ? b->device : 0);
    if (guard.err != hipSuccess) return fail(guard.err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    bst_status st = stage_lists(b, sinos, sino_off, imgs, img_off, ws, ws_bytes, s);
    if (st != BST_OK) return st;
    hipEvent_t t0, t1;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) return fail(e);
    const int slices[4] = {4, 8, 16, 32};
    for (auto& c : b->classes) {
        bst_plan_s& p = *c.plan;
        float best = 1e30f;
        int best_s = p.gather_slices;
        for (int si : slices) {
            p.gather_slices = si;
            e = launch_class(b, c, ws, s);  // warm
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventRecord(t0, s);
            for (int r = 0; e == hipSuccess && r < 2; ++r) e = launch_class(b, c, ws, s);
            if (e == hipSuccess) e = hipEventRecord(t1, s);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e != hipSuccess) break;
            if (ms < best) {
                best = ms;
                best_s = si;
            }
        }
        p.gather_slices = best_s;
        if (e != hipSuccess) break;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return fail(e);
    // a tuned configuration needs a new capture
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    b->graph_ws = nullptr;
    return BST_OK;
}

bst_status bst_batch_backproject(bst_batch_t b, const float* sinos, const int64_t* sino_off, float* imgs,
                                 const int64_t* img_off, void* ws, size_t ws_bytes, void* stream) {
    bst::TraceRange trace("bst_batch_backproject");
    Guard guard(b ? b->device : 0);
    if (guard.err != hipSuccess) return fail(guard.err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    bst_status st = stage_lists(b, sinos, sino_off, imgs, img_off, ws, ws_bytes, s);
    if (st != BST_OK) return st;
    hipError_t e = hipSuccess;
    if (!b->exec || b->graph_ws != ws) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        hipStream_t s0 = b->streams[0];
        e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) e = hipEventRecord(b->fork, s0);
        for (int i = 1; e == hipSuccess && i < kStreams; ++i) e = hipStreamWaitEvent(b->streams[i], b->fork, 0);
        for (size_t k = 0; e == hipSuccess && k < b->classes.size(); ++k)
            e = launch_class(b, b->classes[k], ws, b->streams[k % kStreams]);
        for (int i = 1; e == hipSuccess && i < kStreams; ++i) {
            e = hipEventRecord(b->joins[i], b->streams[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s0, b->joins[i], 0);
        }
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(s0, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(e);
        }
        b->graph = g;
        b->graph_ws = ws;
    }
    e = hipGraphLaunch(b->exec, s);
    return e == hipSuccess ? BST_OK : fail(e);
}

bst_status bst_batch_destroy(bst_batch_t b) {
    release(b);
    return BST_OK;
}

}  // extern "C"
