// batch.cpp -- uneven-size batches: many sinograms of different sizes in one
// graph launch (the paper's pipeline processes blocks of Q sinograms at once,
// Section 3, and Section 4 measures how the block size Q changes its time).
//
// Instances are grouped into size classes of equal n (= N); the angle count V
// may differ per instance. Each class has one plan (the FFT twiddles, taper,
// radial weights of its n, built with the class's largest V) and one
// workspace region laid out for its largest V, one slice per polar group (the
// interleaving of ordinary batches pairs equal angle sets, which instances of
// different V do not have). Per stage and class, one persistent kernel walks
// a device work list of (slice, tile) items, every item carrying its slice's
// own V (the gather reads its angle directions j pi / V from a per-slice
// table built on the host in FP64): spectrum (P1-P4),
// gather + column inverse FFT (P5-P6) and row C2R (P6-P8), plus a sinogram-sum
// kernel with monopole subtraction. Kernels read the instances' sinograms and
// write their images through per-slice pointer lists, so instances need not
// be contiguous or ordered. The first call with a given workspace captures
// every class's launches into one hipGraph, forked over a few streams (all at
// default priority) and joined back; later calls update the pointer lists and
// replay it. bst_batch_tune times, per class and on the caller's data, each
// stage's persistent grid size and the row stage's tile shape (how many row
// tiles one work item covers), and keeps the fastest.
//
// The tent angular rule pre-gathers its patches per angle set, so tent
// batches keep classes of equal (n, V) run by the ordinary kernels (through
// the same pointer lists), one class per pair.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "bst_internal.h"

namespace {

constexpr int kStreams = 4;
constexpr int kStages = 3;  // spectrum, gather, row

struct SizeClass {
    int n = 0, Vmax = 0;
    bool regular = false;      // equal (n, V), ordinary launches (tent rule)
    bst_plan_t plan = nullptr;
    std::vector<int> members;  // instance indices, in input order
    std::vector<int> Vs;       // their angle counts
    int list_base = 0;         // offset of this class's pointers in the lists
    size_t ws_off = 0, ws_bytes = 0;
    // workspace layout (offsets inside the class region)
    size_t polar_off = 0, dc_off = 0, grid_off = 0, mass_off = 0;
    // device arrays (inside the batch's table block): V per slice, work lists
    int* d_V = nullptr;
    int* d_ang_off = nullptr;      // slice i's directions at d_ang + d_ang_off[i]
    const double2* d_ang = nullptr;
    int2* d_items[kStages] = {};
    int n_items[kStages] = {};
    int row_tiles = 1;         // row tiles per item of the row stage (tuned)
    int blocks[kStages] = {};  // persistent grid sizes (tuned)
};

// Work list of a stage: (slice, block) items, slice-major.
std::vector<int2> stage_items(const SizeClass& c, int stage) {
    std::vector<int2> list;
    for (int i = 0; i < (int)c.members.size(); ++i) {
        const int nb = stage == 0 ? bst::spectrum_blocks_per_slice(*c.plan, c.Vs[i])
                                  : (stage == 1 ? bst::gather_blocks_per_slice(*c.plan)
                                                : bst::row_blocks_per_slice(*c.plan, c.row_tiles));
        for (int k = 0; k < nb; ++k) list.push_back(make_int2(i, k));
    }
    return list;
}

// Layout of a class region: polar [B][Vmax][S] complex64 (one slice per
// group), DC terms [B][Vmax], grid [B][N][G/2], monopole sums [B][64].
size_t class_layout(SizeClass& c) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const bst_plan_s& p = *c.plan;
    const size_t B = c.members.size();
    c.polar_off = 0;
    c.dc_off = up(B * (size_t)c.Vmax * p.S * sizeof(float2));
    c.grid_off = up(c.dc_off + B * (size_t)c.Vmax * sizeof(float));
    c.mass_off = up(c.grid_off + B * (size_t)p.N * p.GT * sizeof(float2));
    return up(c.mass_off + (p.monopole ? B * bst::kMassChunks * sizeof(float) : 0));
}

}  // namespace

struct bst_batch_s {
    int device = 0;
    int count = 0;
    int cus = 0;                          // compute units of the device
    std::vector<SizeClass> classes;
    size_t ws_total = 0;
    void* d_lists = nullptr;              // device: [count] sinogram then [count] image pointers
    const float** d_sino_list = nullptr;
    float** d_img_list = nullptr;
    void* h_lists = nullptr;              // pinned host staging, 2 * count pointers
    hipEvent_t lists_done = nullptr;      // the staging may be rewritten after this
    void* d_tables = nullptr;             // per-slice V and work lists of every class
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
    if (b->d_tables) (void)hipFree(b->d_tables);
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

// Enqueue a regular class (equal n and V) on `st`: the ordinary kernels, as
// for a batch of one plan, reading and writing through the pointer lists.
hipError_t launch_regular(const bst_batch_s* b, const SizeClass& c, void* ws, hipStream_t st) {
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
    const float* const* sinos = b->d_sino_list + c.list_base;
    hipError_t e;
    if (p.monopole) {
        const bst::MassArgs ma{nullptr, sinos, nullptr, nullptr, mass, p.n, p.V};
        e = bst::launch_mass(p, ma, batch, st);
        if (e != hipSuccess) return e;
    }
    const bst::SpecArgs sa{nullptr, sinos, nullptr, nullptr, polar, dc, p.taper, p.kc, p.tw_M, p.n, p.V, p.S,
                           p.lead, p.S - p.lead - p.M / 2, (float)p.dt, mass, p.mono_phi, p.mono_inv};
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
    const bst::RowArgs ra{grid, nullptr, b->d_img_list + c.list_base, p.tw_G, p.N, p.GT, p.out_scale, 0,
                          mass, p.mono_inv, p.mono_amp, p.mono_rho_px};
    return bst::launch_row_c2r(p, ra, batch, st);
}

// Enqueue one class's stages on `st`: the persistent spectrum, gather and row
// kernels (and the monopole sums first).
hipError_t launch_class(const bst_batch_s* b, const SizeClass& c, void* ws, hipStream_t st) {
    if (c.regular) return launch_regular(b, c, ws, st);
    const bst_plan_s& p = *c.plan;
    const int batch = (int)c.members.size();
    unsigned char* w = static_cast<unsigned char*>(ws) + c.ws_off;
    float2* polar = reinterpret_cast<float2*>(w + c.polar_off);
    float* dc = reinterpret_cast<float*>(w + c.dc_off);
    float2* grid = reinterpret_cast<float2*>(w + c.grid_off);
    float* mass = p.monopole ? reinterpret_cast<float*>(w + c.mass_off) : nullptr;
    const float* const* sinos = b->d_sino_list + c.list_base;
    hipError_t e;
    if (p.monopole) {
        bst::MassArgs ma{nullptr, sinos, nullptr, nullptr, mass, p.n, c.Vmax, c.d_V};
        e = bst::launch_mass(p, ma, batch, st);
        if (e != hipSuccess) return e;
    }
    bst::SpecArgs sa{nullptr, sinos, nullptr, nullptr, polar, dc, p.taper, p.kc, p.tw_M, p.n, c.Vmax, p.S, p.lead,
                     p.S - p.lead - p.M / 2, (float)p.dt, mass, p.mono_phi, p.mono_inv};
    sa.Vs = c.d_V;
    sa.items = c.d_items[0];
    sa.n_items = c.n_items[0];
    e = bst::launch_spectrum_items(p, sa, batch, c.blocks[0], st);
    if (e != hipSuccess) return e;
    bst::GatherArgs ga{};
    ga.polar = polar;
    ga.dc = dc;
    ga.grid = grid;
    ga.tw = p.tw_G;
    ga.V = c.Vmax;
    ga.S = p.S;
    ga.GT = p.GT;
    ga.N = p.N;
    ga.Mh = p.M / 2;
    ga.zero_slot = p.M / 2 + p.lead;
    ga.uniform = 1;
    ga.batch = batch;
    ga.slices_per_block = 1;
    ga.rscale = p.rscale;
    ga.dc_rule = p.dc_scale * (float)p.V;  // the plan's per-projection factor times its V
    ga.Vs = c.d_V;
    ga.ang = c.d_ang;
    ga.ang_off = c.d_ang_off;
    ga.items = c.d_items[1];
    ga.n_items = c.n_items[1];
    e = bst::launch_gather_items(p, ga, c.blocks[1], st);
    if (e != hipSuccess) return e;
    bst::RowArgs ra{grid, nullptr, b->d_img_list + c.list_base, p.tw_G, p.N, p.GT, p.out_scale, c.row_tiles,
                    mass, p.mono_inv, p.mono_amp, p.mono_rho_px};
    ra.V = p.V;
    ra.Vs = c.d_V;
    ra.items = c.d_items[2];
    ra.n_items = c.n_items[2];
    return bst::launch_row_items(p, ra, c.blocks[2], st);
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

// the persistent grid of a stage: k blocks per compute unit, at most one per item
int grid_blocks(const bst_batch_s* b, int items, int per_cu) {
    return std::max(1, std::min(items, per_cu * b->cus));
}

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
    const bool regular = base->angular == BST_ANGULAR_TENT;
    std::map<std::pair<int, int>, int> index;  // (n, V or 0) -> class
    std::vector<SizeClass> classes;
    for (int i = 0; i < count; ++i) {
        bst_params p = *base;
        p.n_det = n_det[i];
        p.n_out = n_det[i];
        p.n_angles = n_angles[i];
        p.max_batch = 1;
        const bst_status st = bst_validate(&p);
        if (st != BST_OK) return st;
        const auto key = std::make_pair((int)n_det[i], regular ? (int)n_angles[i] : 0);
        auto it = index.find(key);
        if (it == index.end()) {
            it = index.emplace(key, (int)classes.size()).first;
            classes.emplace_back();
            classes.back().n = n_det[i];
            classes.back().regular = regular;
        }
        SizeClass& c = classes[it->second];
        c.members.push_back(i);
        c.Vs.push_back(n_angles[i]);
        c.Vmax = std::max(c.Vmax, (int)n_angles[i]);
    }
    bst_batch_s* b = new (std::nothrow) bst_batch_s();
    if (!b) return BST_E_NOMEM;
    b->device = base->device;
    b->count = count;
    b->classes = std::move(classes);
    Guard guard(b->device);
    if (guard.err != hipSuccess) {
        delete b;
        return fail(guard.err);
    }
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, b->device);
    if (e != hipSuccess) {
        delete b;
        return fail(e);
    }
    b->cus = prop.multiProcessorCount;
    int list_base = 0;
    size_t off = 0;
    std::vector<std::vector<int2>> items;  // per class and stage
    for (auto& c : b->classes) {
        bst_params p = *base;
        p.n_det = c.n;
        p.n_out = c.n;
        p.n_angles = c.Vmax;
        p.max_batch = (int32_t)c.members.size();
        p.adjoint = 0;
        const bst_status st = bst_plan(&p, &c.plan);
        if (st != BST_OK) {
            release(b);
            return st;
        }
        c.list_base = list_base;
        list_base += (int)c.members.size();
        c.ws_off = off;
        if (c.regular) {
            (void)bst_workspace_size(c.plan, p.max_batch, &c.ws_bytes);
            off += (c.ws_bytes + 255) & ~(size_t)255;
            for (int s = 0; s < kStages; ++s) items.emplace_back();
            continue;
        }
        c.ws_bytes = class_layout(c);
        off += c.ws_bytes;
        // work lists; the row list's region holds the finest tiling (one tile
        // per item), which the tuner may pick. Start with about four row
        // blocks per compute unit.
        const int B = (int)c.members.size();
        const int per_slice = bst::row_blocks_per_slice(*c.plan, 1);
        c.row_tiles = std::max(1, std::min(bst::row_max_tiles(*c.plan), (per_slice * B) / (4 * b->cus)));
        for (int s = 0; s < kStages; ++s) {
            std::vector<int2> list = stage_items(c, s);
            c.n_items[s] = (int)list.size();
            if (s == 2) list.resize((size_t)per_slice * B, make_int2(0, 0));
            items.push_back(std::move(list));
        }
        c.blocks[0] = grid_blocks(b, c.n_items[0], 2);
        c.blocks[1] = grid_blocks(b, c.n_items[1], 1);
        c.blocks[2] = grid_blocks(b, c.n_items[2], 2);
    }
    b->ws_total = off;
    // one device block: per class its V list, the offsets of its slices'
    // direction tables, the tables ((cos, sin) of j pi / V_i, in FP64 as for
    // a plan), then its three work lists
    auto up16 = [](size_t x) { return (x + 15) / 16 * 16; };
    size_t tbytes = 0;
    std::vector<size_t> v_off(b->classes.size()), a_off(b->classes.size()), d_off(b->classes.size()),
        i_off(b->classes.size() * kStages);
    for (size_t k = 0; k < b->classes.size(); ++k) {
        const SizeClass& c = b->classes[k];
        v_off[k] = tbytes;
        tbytes += up16(c.members.size() * sizeof(int));
        a_off[k] = tbytes;
        tbytes += up16(c.members.size() * sizeof(int));
        d_off[k] = tbytes;
        size_t dirs = 0;
        for (int V : c.Vs) dirs += (size_t)V;
        if (dirs > (size_t)INT32_MAX) {  // the slices' table offsets are 32-bit
            release(b);
            return BST_E_BATCH;
        }
        tbytes += dirs * sizeof(double2);
        for (int s = 0; s < kStages; ++s) {
            i_off[k * kStages + s] = tbytes;
            tbytes += std::max<size_t>(items[k * kStages + s].size(), 1) * sizeof(int2);
        }
    }
    std::vector<unsigned char> host(tbytes, 0);
    for (size_t k = 0; k < b->classes.size(); ++k) {
        const SizeClass& c = b->classes[k];
        int first = 0;  // direction-table offset of slice i, in entries
        for (size_t i = 0; i < c.members.size(); ++i) {
            const int V = n_angles[c.members[i]];
            std::memcpy(host.data() + v_off[k] + i * sizeof(int), &V, sizeof(int));
            std::memcpy(host.data() + a_off[k] + i * sizeof(int), &first, sizeof(int));
            for (int j = 0; j < V; ++j) {
                const double th = (double)j * M_PI / (double)V;
                const double2 d = make_double2(std::cos(th), std::sin(th));
                std::memcpy(host.data() + d_off[k] + (size_t)(first + j) * sizeof(double2), &d, sizeof(double2));
            }
            first += V;
        }
        for (int s = 0; s < kStages; ++s) {
            const auto& l = items[k * kStages + s];
            if (!l.empty()) std::memcpy(host.data() + i_off[k * kStages + s], l.data(), l.size() * sizeof(int2));
        }
    }
    e = hipMalloc(&b->d_tables, std::max<size_t>(tbytes, 16));
    if (e == hipSuccess) e = hipMemcpy(b->d_tables, host.data(), tbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&b->d_lists, 2 * (size_t)count * sizeof(void*));
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
    unsigned char* tb = static_cast<unsigned char*>(b->d_tables);
    for (size_t k = 0; k < b->classes.size(); ++k) {
        SizeClass& c = b->classes[k];
        c.d_V = reinterpret_cast<int*>(tb + v_off[k]);
        c.d_ang_off = reinterpret_cast<int*>(tb + a_off[k]);
        c.d_ang = reinterpret_cast<const double2*>(tb + d_off[k]);
        for (int s = 0; s < kStages; ++s) c.d_items[s] = reinterpret_cast<int2*>(tb + i_off[k * kStages + s]);
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
    // the row stage's work list for a tiling (synchronous upload: every
    // launch that read the previous list has finished)
    auto set_row_tiles = [&](SizeClass& c, int tiles) {
        c.row_tiles = tiles;
        const std::vector<int2> list = stage_items(c, 2);
        c.n_items[2] = (int)list.size();
        hipError_t r = hipStreamSynchronize(s);
        if (r == hipSuccess) r = hipMemcpy(c.d_items[2], list.data(), list.size() * sizeof(int2), hipMemcpyHostToDevice);
        return r;
    };
    // per class, stage by stage: the persistent grid (blocks per compute unit)
    // and, for the row stage, the tiles per item with which the class's
    // launches run fastest on these inputs
    const int per_cu[4] = {1, 2, 4, 8};
    for (auto& c : b->classes) {
        for (int stage = 0; !c.regular && stage < kStages && e == hipSuccess; ++stage) {
            float best = 1e30f;
            int best_blocks = c.blocks[stage], best_tiles = c.row_tiles;
            const int max_tiles = stage == 2 ? bst::row_max_tiles(*c.plan) : 1;
            for (int tiles = 1; tiles <= max_tiles && e == hipSuccess; tiles *= 2) {
                if (stage == 2) e = set_row_tiles(c, tiles);
                int tried = -1;
                for (int k : per_cu) {
                    if (e != hipSuccess) break;
                    const int blocks = grid_blocks(b, c.n_items[stage], k);
                    if (blocks == tried) continue;  // capped by the item count
                    tried = blocks;
                    c.blocks[stage] = blocks;
                    e = launch_class(b, c, ws, s);  // warm
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventRecord(t0, s);
                    for (int r = 0; e == hipSuccess && r < 2; ++r) e = launch_class(b, c, ws, s);
                    if (e == hipSuccess) e = hipEventRecord(t1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(t1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                    if (e == hipSuccess && ms < best) {
                        best = ms;
                        best_blocks = blocks;
                        best_tiles = tiles;
                    }
                }
            }
            if (e == hipSuccess && stage == 2) e = set_row_tiles(c, best_tiles);
            c.blocks[stage] = best_blocks;
        }
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
