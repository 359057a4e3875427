// C-ABI entry points of the neuda library: argument validation, device
// memory ownership, host/device staging and error translation.  Every
// numeric step runs in the kernels of the .hip files.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nd_internal.h"

// Scratch of nd_forces_noalloc: a fixed array in every GPU's memory, sized
// for ND_NOALLOC_MAX_ATOMS atoms and a grid of at most NOALLOC_MAX_GRID
// blocks, plus a sink for an energy the caller does not want.  In host code
// `scratch` names a host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
namespace {
constexpr long long NOALLOC_MAX_GRID = 2048;
constexpr size_t NOALLOC_FORCES_BYTES =
    sizeof(long long) * 2 * 3 * (size_t)ND_NOALLOC_MAX_ATOMS + sizeof(double) * NOALLOC_MAX_GRID + 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_FORCES_BYTES + 256;
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
thread_local std::string g_last_error;

nd_status set_error(nd_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

template <class F>
nd_status guarded(F &&f)
{
    try {
        g_last_error.clear();
        f();
        return ND_OK;
    } catch (const nd::Error &e) {
        return set_error(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return set_error(ND_E_OOM, "host allocation failed");
    } catch (...) {
        return set_error(ND_E_INVALID, "unexpected internal error");
    }
}

void require(bool cond, nd_status code, const std::string &msg)
{
    if (!cond) nd::fail(code, msg);
}

void check_where(int32_t where)
{
    require(where == ND_HOST || where == ND_DEVICE, ND_E_INVALID, "where must be ND_HOST or ND_DEVICE");
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ND_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Temporary device buffer freed at scope exit (after the stream drains).
struct Scratch {
    void *p = nullptr;
    hipStream_t s = nullptr;
    Scratch(size_t bytes, hipStream_t st) : s(st) { p = nd::dmalloc(bytes); }
    ~Scratch()
    {
        if (p) {
            (void)hipStreamSynchronize(s);
            nd::dfree(p);
        }
    }
    template <class T>
    T *as() { return static_cast<T *>(p); }
};

void validate_xyz_host(const float *xyz, int N, double L)
{
    for (size_t i = 0; i < (size_t)3 * N; ++i) {
        float v = xyz[i];
        require(std::isfinite(v), ND_E_INVALID, "coordinate is not finite");
        require(v >= 0.0f && (double)v < L, ND_E_INVALID, "coordinate outside [0, L)");
    }
}

void check_box(nd_box *b)
{
    require(b != nullptr, ND_E_INVALID, "box is NULL");
}

void check_mc_params(const nd_box *b, const nd_mc_params *p)
{
    require(p != nullptr, ND_E_INVALID, "params is NULL");
    require(std::isfinite(p->kT) && p->kT > 0.0, ND_E_INVALID, "kT must be > 0");
    require(std::isfinite(p->max_disp) && p->max_disp >= 0.0, ND_E_INVALID, "max_disp must be >= 0");
    require(std::isfinite(p->max_rot) && p->max_rot >= 0.0, ND_E_INVALID, "max_rot must be >= 0");
    require(p->max_disp < 0.25 * b->L, ND_E_RANGE, "max_disp must be < L/4");
    require(p->tie_rel >= 0.0 && std::isfinite(p->tie_rel), ND_E_INVALID, "tie_rel must be >= 0");
    require(p->k_batch >= 0, ND_E_INVALID, "k_batch must be >= 0");
    require(p->order == ND_ORDER_SEQ || p->order == ND_ORDER_RANDOM, ND_E_INVALID, "unknown order");
    require(p->scan == ND_SCAN_CELLS || p->scan == ND_SCAN_FULL, ND_E_INVALID, "unknown scan mode");
    require(std::isfinite(p->atom_frac) && p->atom_frac >= 0.0 && p->atom_frac <= 1.0, ND_E_INVALID,
            "atom_frac must be in [0, 1]");
    require(std::isfinite(p->atom_disp) && p->atom_disp >= 0.0, ND_E_INVALID, "atom_disp must be >= 0");
    require(p->atom_disp < 0.25 * b->L, ND_E_RANGE, "atom_disp must be < L/4");
    require(b->has_tables, ND_E_STATE, "nd_box_set_tables has not been called");
}

void check_hist_range(const nd_box *b, double dr, int32_t nbins)
{
    require(std::isfinite(dr) && dr > 0.0, ND_E_INVALID, "dr must be > 0");
    require(nbins >= 1, ND_E_INVALID, "nbins must be >= 1");
    require((double)nbins * dr < 0.5 * b->L * (1.0 - 1e-9), ND_E_RANGE, "nbins*dr must be < L/2");
}

void box_npairs(const nd_box *b, double *npairs)
{
    for (int a = 0; a < b->M; ++a)
        for (int c = a; c < b->M; ++c) {
            const double na = (double)b->species_count[a], nc = (double)b->species_count[c];
            npairs[nd::pair_index(a, c, b->M)] = (a == c) ? na * (na - 1.0) / 2.0 : na * nc;
        }
}

// ---- checkpoint image (nd_box_save / nd_box_load)
// Little-endian layout: a fixed header, then the coordinates and, when the
// cell lists are live, their slot order, start table and rebuild
// positions, and last an FNV-1a 64-bit hash of everything before it.
constexpr char CKPT_MAGIC[8] = {'N', 'D', 'B', 'O', 'X', 'C', 'K', '1'};

struct CkptHeader {
    char magic[8];
    int32_t version, n_atoms, n_species, n_units;
    double L;
    double E;
    int32_t energy_valid, cells_valid, nc, ncell;
    int64_t trials_since_build;
    float drift;
    int32_t pad;
};

uint64_t fnv1a(const unsigned char *p, size_t n)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

size_t ckpt_size(const nd_box *b, bool cells, int ncell)
{
    size_t n = sizeof(CkptHeader) + sizeof(float) * 3 * (size_t)b->N;
    if (cells) n += sizeof(int32_t) * 2 * (size_t)b->N + sizeof(int32_t) * (size_t)(ncell + 1) +
                    sizeof(float4) * (size_t)b->N;
    return n + sizeof(uint64_t);
}

std::mutex g_tune_mu;
std::vector<nd_tuning> g_tune;

void check_tuning(const nd_tuning &e)
{
    require(e.kind == ND_TUNE_BOX || e.kind == ND_TUNE_BATCH, ND_E_INVALID, "tuning kind must be box or batch");
    require(e.scan_waves == 0 || e.scan_waves == 1 || e.scan_waves == 2 || e.scan_waves == 4, ND_E_INVALID,
            "scan_waves must be 0, 1, 2 or 4");
    require(std::isfinite(e.batch_target) && e.batch_target >= 0.0, ND_E_INVALID, "batch_target must be >= 0");
    require(e.hist_blocks_per_cu >= 0 && e.hist_blocks_per_cu <= 8, ND_E_INVALID,
            "hist_blocks_per_cu must be in 0..8");
    require(e.n_max >= 0, ND_E_INVALID, "n_max must be >= 0");
}

}  // namespace

namespace nd {

bool tune_lookup(int kind, long long n, nd_tuning *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const nd_tuning &e : g_tune)
        if (e.kind == kind && n <= e.n_max) {
            *out = e;
            return true;
        }
    return false;
}

[[noreturn]] void fail(nd_status code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(ND_E_OOM, std::string("device allocation failed: ") + what);
    fail(ND_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void *dmalloc(size_t bytes)
{
    if (bytes == 0) bytes = 16;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (e == hipErrorOutOfMemory) fail(ND_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        fail(ND_E_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return p;
}

void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

void *workspace(nd_box *b, size_t bytes)
{
    if (bytes <= b->ws_bytes && b->ws) return b->ws;
    ND_HIP(hipStreamSynchronize(b->stream));
    dfree(b->ws);
    b->ws = nullptr;
    b->ws_bytes = 0;
    size_t cap = bytes + bytes / 4;
    b->ws = dmalloc(cap);
    b->ws_bytes = cap;
    return b->ws;
}

int cu_count(int device)
{
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
    return n;
}

static hipEvent_t take_event(nd_box *b)
{
    if (!b->prof_free.empty()) {
        hipEvent_t e = b->prof_free.back();
        b->prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    ND_HIP(hipEventCreate(&e));
    return e;
}

ProfScope::ProfScope(nd_box *box, int k) : b(box), kind(k)
{
    if (kind < 0 || !(b->prof_mask & (1u << kind))) return;
    if (b->prof_pending[kind].size() >= 8192) prof_harvest(b);
    e1 = take_event(b);
    e2 = take_event(b);
    ND_HIP(hipEventRecord(e1, b->stream));
}

ProfScope::~ProfScope()
{
    if (!e1) return;
    if (hipEventRecord(e2, b->stream) == hipSuccess) {
        b->prof_pending[kind].emplace_back(e1, e2);
    } else {
        b->prof_free.push_back(e1);
        b->prof_free.push_back(e2);
    }
}

void prof_harvest(nd_box *b)
{
    ND_HIP(hipStreamSynchronize(b->stream));
    for (int k = 0; k < ND_PROF_KINDS; ++k) {
        for (auto &pr : b->prof_pending[k]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
                b->prof_ms[k] += ms;
                b->prof_n[k] += 1;
            }
            b->prof_free.push_back(pr.first);
            b->prof_free.push_back(pr.second);
        }
        b->prof_pending[k].clear();
    }
}

void prof_release(nd_box *b)
{
    for (int k = 0; k < ND_PROF_KINDS; ++k) {
        for (auto &pr : b->prof_pending[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        b->prof_pending[k].clear();
    }
    for (auto e : b->prof_free) (void)hipEventDestroy(e);
    b->prof_free.clear();
}

}  // namespace nd

static void free_box(nd_box *b)
{
    if (!b) return;
    nd::prof_release(b);
    nd::dfree(b->xyz);
    nd::dfree(b->pos4);
    nd::dfree(b->poslo);
    nd::dfree(b->species);
    nd::dfree(b->uoff);
    nd::dfree(b->unit_of);
    nd::dfree(b->tab);
    nd::dfree(b->rp);
    nd::dfree(b->emp);
    nd::dfree(b->r0);
    nd::dfree(b->scan_count);
    nd::dfree(b->E);
    nd::dfree(b->mc.trials);
    nd::dfree(b->mc.partial);
    nd::dfree(b->mc.corr_n);
    nd::dfree(b->mc.corr_ptr);
    nd::dfree(b->mc.ovf_fill);
    nd::dfree(b->mc.counters);
    nd::dfree(b->mc.dsum);
    nd::dfree(b->mc.pool_m);
    nd::dfree(b->mc.pool_c);
    nd::dfree(b->mc.corr_s);
    nd::dfree(b->mc.corr_b);
    nd::dfree(b->mc.spheres);
    nd::dfree(b->mc.head);
    nd::dfree(b->mc.hthr);
    nd::dfree(b->mc.dE0);
    nd::dfree(b->mc.S0);
    nd::dfree(b->mc.thr);
    nd::dfree(b->bt_dev);
    nd::dfree(b->mc.acc_flags);
    nd::cells_free(b);
    nd::dfree(b->track.counts);
    nd::dfree(b->track.sum);
    nd::dfree(b->track.partial);
    nd::dfree(b->track.moved);
    nd::dfree(b->ws);
    delete[] b->h_uoff;
    delete[] b->h_species;
    delete b;
}

// Several boxes run as one graph of launches (the batched form).
struct nd_batch {
    std::vector<nd_box *> boxes;
    int device = 0;
    hipStream_t stream = nullptr;  // owned; graphs are captured and replayed on it
    hipEvent_t ev_done = nullptr;
    std::vector<hipEvent_t> ev_in;  // one per box
    nd::McMulti *mc = nullptr;
    nd::HistMulti *hist = nullptr;
    nd::SqMulti *sq = nullptr;
    std::vector<long long> sig;     // launch structure of the captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    long long captures = 0, launches = 0;
};

static void free_batch(nd_batch *t)
{
    if (!t) return;
    if (t->stream) (void)hipStreamSynchronize(t->stream);
    if (t->exec) (void)hipGraphExecDestroy(t->exec);
    if (t->graph) (void)hipGraphDestroy(t->graph);
    nd::mc_multi_destroy(t->mc);
    nd::hist_multi_destroy(t->hist);
    nd::sq_multi_destroy(t->sq);
    for (auto e : t->ev_in) (void)hipEventDestroy(e);
    if (t->ev_done) (void)hipEventDestroy(t->ev_done);
    if (t->stream) (void)hipStreamDestroy(t->stream);
    delete t;
}

extern "C" {

int32_t nd_abi_version(void) { return ND_ABI_VERSION; }

const char *nd_last_error(void) { return g_last_error.c_str(); }

nd_status nd_box_create(const nd_box_desc *d, nd_box **out)
{
    return guarded([&] {
        require(d != nullptr && out != nullptr, ND_E_INVALID, "desc or out is NULL");
        *out = nullptr;
        require(d->n_atoms >= 2, ND_E_INVALID, "n_atoms must be >= 2");
        require(d->n_species >= 1 && d->n_species <= ND_MAX_SPECIES, ND_E_INVALID,
                "n_species must be in 1..ND_MAX_SPECIES");
        require(std::isfinite(d->L) && d->L > 0.0, ND_E_INVALID, "L must be finite and > 0");
        require(d->species && d->unit_offsets && d->xyz, ND_E_INVALID, "species, unit_offsets and xyz are required");
        require(d->n_units >= 1 && d->n_units <= d->n_atoms, ND_E_INVALID, "n_units out of range");
        const int N = d->n_atoms;
        require(d->unit_offsets[0] == 0 && d->unit_offsets[d->n_units] == N, ND_E_INVALID,
                "unit_offsets must start at 0 and end at n_atoms");
        int max_na = 0;
        for (int u = 0; u < d->n_units; ++u) {
            int na = d->unit_offsets[u + 1] - d->unit_offsets[u];
            require(na >= 1, ND_E_INVALID, "unit_offsets must be strictly increasing");
            require(na <= ND_MAX_UNIT_ATOMS, ND_E_INVALID, "unit larger than ND_MAX_UNIT_ATOMS atoms");
            if (na > max_na) max_na = na;
        }
        int64_t cnt[ND_MAX_SPECIES] = {0, 0, 0, 0};
        for (int i = 0; i < N; ++i) {
            require(d->species[i] < d->n_species, ND_E_INVALID, "species index >= n_species");
            cnt[d->species[i]]++;
        }
        validate_xyz_host(d->xyz, N, d->L);

        DeviceGuard g(d->device);
        nd_box *b = new nd_box();
        try {
            b->device = d->device;
            b->stream = static_cast<hipStream_t>(d->stream);
            b->N = N;
            b->M = d->n_species;
            b->P = d->n_species * (d->n_species + 1) / 2;
            b->n_units = d->n_units;
            b->max_na = max_na;
            b->L = d->L;
            for (int s = 0; s < ND_MAX_SPECIES; ++s) b->species_count[s] = cnt[s];
            b->h_uoff = new int32_t[d->n_units + 1];
            std::memcpy(b->h_uoff, d->unit_offsets, sizeof(int32_t) * (d->n_units + 1));
            b->h_species = new uint8_t[N];
            std::memcpy(b->h_species, d->species, N);
            std::vector<int32_t> unit_of(N);
            for (int u = 0; u < d->n_units; ++u)
                for (int a = d->unit_offsets[u]; a < d->unit_offsets[u + 1]; ++a) unit_of[a] = u;

            b->xyz = static_cast<float *>(nd::dmalloc(sizeof(float) * 3 * (size_t)N));
            b->pos4 = static_cast<float4 *>(nd::dmalloc(sizeof(float4) * (size_t)N));
            b->poslo = static_cast<float4 *>(nd::dmalloc(sizeof(float4) * (size_t)N));
            b->species = static_cast<uint8_t *>(nd::dmalloc((size_t)N));
            b->uoff = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * (d->n_units + 1)));
            b->unit_of = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * (size_t)N));
            b->E = static_cast<double *>(nd::dmalloc(sizeof(double)));
            ND_HIP(hipMemcpyAsync(b->xyz, d->xyz, sizeof(float) * 3 * (size_t)N, hipMemcpyHostToDevice, b->stream));
            ND_HIP(hipMemcpyAsync(b->species, d->species, (size_t)N, hipMemcpyHostToDevice, b->stream));
            ND_HIP(hipMemcpyAsync(b->uoff, d->unit_offsets, sizeof(int32_t) * (d->n_units + 1),
                                  hipMemcpyHostToDevice, b->stream));
            ND_HIP(hipMemcpyAsync(b->unit_of, unit_of.data(), sizeof(int32_t) * (size_t)N,
                                  hipMemcpyHostToDevice, b->stream));
            ND_HIP(hipMemsetAsync(b->E, 0, sizeof(double), b->stream));
            nd::launch_pos4_from_xyz(b);
            ND_HIP(hipStreamSynchronize(b->stream));
        } catch (...) {
            free_box(b);
            throw;
        }
        *out = b;
    });
}

nd_status nd_box_destroy(nd_box *b)
{
    return guarded([&] {
        if (!b) return;
        // When the HIP runtime is no longer usable (a destroy reached during
        // process teardown) the device memory goes with the process; only
        // the host side is released.
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(b->device) != hipSuccess) {
            (void)hipGetLastError();
            delete[] b->h_uoff;
            delete[] b->h_species;
            delete b;
            return;
        }
        (void)hipStreamSynchronize(b->stream);
        free_box(b);
        if (prev >= 0) (void)hipSetDevice(prev);
    });
}

nd_status nd_box_set_profiling_mask(nd_box *b, uint32_t kernels)
{
    return guarded([&] {
        check_box(b);
        require((kernels >> ND_PROF_KINDS) == 0, ND_E_INVALID, "unknown kernel bit");
        DeviceGuard g(b->device);
        nd::prof_harvest(b);
        if (kernels) {
            for (int k = 0; k < ND_PROF_KINDS; ++k) {
                b->prof_ms[k] = 0.0;
                b->prof_n[k] = 0;
            }
        }
        b->prof_mask = kernels;
    });
}

nd_status nd_box_set_profiling(nd_box *b, int32_t enable)
{
    return nd_box_set_profiling_mask(b, enable ? (1u << ND_PROF_KINDS) - 1u : 0u);
}

nd_status nd_box_count_scan(nd_box *b, int32_t enable, int64_t *candidates, int64_t *survivors)
{
    return guarded([&] {
        check_box(b);
        DeviceGuard g(b->device);
        if (b->scan_count) {
            unsigned long long c[2];
            ND_HIP(hipMemcpyAsync(c, b->scan_count, sizeof(c), hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
            if (candidates) *candidates = (int64_t)c[0];
            if (survivors) *survivors = (int64_t)c[1];
        } else {
            if (candidates) *candidates = 0;
            if (survivors) *survivors = 0;
        }
        if (enable) {
            if (!b->scan_count) b->scan_count = static_cast<unsigned long long *>(nd::dmalloc(2 * sizeof(unsigned long long)));
            ND_HIP(hipMemsetAsync(b->scan_count, 0, 2 * sizeof(unsigned long long), b->stream));
        } else {
            ND_HIP(hipStreamSynchronize(b->stream));
            nd::dfree(b->scan_count);
            b->scan_count = nullptr;
        }
    });
}

nd_status nd_box_profile(nd_box *b, int32_t kernel, int64_t *launches, double *ms)
{
    return guarded([&] {
        check_box(b);
        require(kernel >= 0 && kernel < ND_PROF_KINDS, ND_E_INVALID, "unknown kernel id");
        require(launches && ms, ND_E_INVALID, "NULL argument");
        DeviceGuard g(b->device);
        nd::prof_harvest(b);
        *launches = b->prof_n[kernel];
        *ms = b->prof_ms[kernel];
    });
}

nd_status nd_box_set_stream(nd_box *b, void *stream)
{
    return guarded([&] {
        check_box(b);
        b->stream = static_cast<hipStream_t>(stream);
    });
}

nd_status nd_box_set_coords(nd_box *b, const float *xyz, int32_t where, int32_t keep_energy)
{
    return guarded([&] {
        check_box(b);
        require(xyz != nullptr, ND_E_INVALID, "xyz is NULL");
        check_where(where);
        DeviceGuard g(b->device);
        size_t bytes = sizeof(float) * 3 * (size_t)b->N;
        if (where == ND_HOST) {
            validate_xyz_host(xyz, b->N, b->L);
            ND_HIP(hipMemcpyAsync(b->xyz, xyz, bytes, hipMemcpyHostToDevice, b->stream));
            nd::launch_pos4_from_xyz(b);
            ND_HIP(hipStreamSynchronize(b->stream));
        } else {
            // wrapped and checked in a staging copy, so that rejected input
            // leaves the box unchanged
            char *stage = static_cast<char *>(nd::workspace(b, bytes + 256));
            int *bad = reinterpret_cast<int *>(stage + bytes);
            ND_HIP(hipMemsetAsync(bad, 0, sizeof(int), b->stream));
            nd::launch_wrap_coords(b, xyz, reinterpret_cast<float *>(stage), bad);
            int h_bad = 0;
            ND_HIP(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
            require(h_bad == 0, ND_E_INVALID, "coordinate is not finite");
            ND_HIP(hipMemcpyAsync(b->xyz, stage, bytes, hipMemcpyDeviceToDevice, b->stream));
            nd::launch_pos4_from_xyz(b);
        }
        if (!keep_energy) b->energy_valid = false;
        b->cells.valid = false;
        b->track.valid = false;
    });
}

nd_status nd_box_get_coords(nd_box *b, float *xyz, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(xyz != nullptr, ND_E_INVALID, "xyz is NULL");
        check_where(where);
        DeviceGuard g(b->device);
        size_t bytes = sizeof(float) * 3 * (size_t)b->N;
        if (where == ND_HOST) {
            ND_HIP(hipMemcpyAsync(xyz, b->xyz, bytes, hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
        } else {
            ND_HIP(hipMemcpyAsync(xyz, b->xyz, bytes, hipMemcpyDeviceToDevice, b->stream));
        }
    });
}

nd_status nd_box_set_tables(nd_box *b, const float *U, int32_t n_pts, double h, double r_cut)
{
    return guarded([&] {
        check_box(b);
        require(U != nullptr, ND_E_INVALID, "U is NULL");
        require(std::isfinite(h) && h > 0.0, ND_E_INVALID, "h must be > 0");
        require(std::isfinite(r_cut) && r_cut > 0.0, ND_E_INVALID, "r_cut must be > 0");
        require(r_cut <= 0.5 * b->L, ND_E_RANGE, "r_cut must be <= L/2");
        require(n_pts >= 2 && (double)(n_pts - 1) * h >= r_cut * (1.0 - 1e-12), ND_E_INVALID,
                "n_pts must satisfy (n_pts - 1) h >= r_cut");
        require(n_pts <= 16384, ND_E_INVALID, "n_pts larger than 16384");
        size_t cnt = (size_t)b->P * n_pts;
        for (size_t i = 0; i < cnt; ++i) require(std::isfinite(U[i]), ND_E_INVALID, "table value is not finite");
        DeviceGuard g(b->device);
        float *t = static_cast<float *>(nd::dmalloc(sizeof(float) * cnt));
        float *r = nullptr;
        try {
            r = static_cast<float *>(nd::dmalloc(sizeof(float) * cnt));
        } catch (...) {
            nd::dfree(t);
            throw;
        }
        hipError_t e = hipMemcpyAsync(t, U, sizeof(float) * cnt, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(r, U, sizeof(float) * cnt, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) {
            nd::dfree(t);
            nd::dfree(r);
            nd::check_hip(e, "copy tables");
        }
        nd::dfree(b->tab);
        nd::dfree(b->rp);
        nd::dfree(b->emp);  // a new reference potential starts without EMP
        b->emp = nullptr;
        b->tab = t;
        b->rp = r;
        b->n_pts = n_pts;
        b->h = h;
        b->rc = r_cut;
        b->has_tables = true;
        b->energy_valid = false;
    });
}

nd_status nd_box_total_energy(nd_box *b, double *E)
{
    return guarded([&] {
        check_box(b);
        require(E != nullptr, ND_E_INVALID, "E is NULL");
        require(b->has_tables, ND_E_STATE, "nd_box_set_tables has not been called");
        DeviceGuard g(b->device);
        nd::launch_total_energy(b, b->E, nullptr);
        nd::launch_intra_energy_add(b, b->E, nullptr);
        ND_HIP(hipMemcpyAsync(E, b->E, sizeof(double), hipMemcpyDeviceToHost, b->stream));
        ND_HIP(hipStreamSynchronize(b->stream));
        b->energy_valid = true;
    });
}

nd_status nd_box_set_intra(nd_box *b, const double *k)
{
    return guarded([&] {
        check_box(b);
        if (k)
            for (int p = 0; p < b->P; ++p)
                require(std::isfinite(k[p]) && k[p] >= 0.0, ND_E_INVALID, "k must be finite and >= 0");
        DeviceGuard g(b->device);
        if (!k) {
            b->has_intra = false;
            for (double &v : b->kint) v = 0.0;
        } else {
            for (int p = 0; p < b->P; ++p) b->kint[p] = k[p];
            nd::launch_intra_reference(b);
            b->has_intra = true;
        }
        b->energy_valid = false;
    });
}

nd_status nd_box_energy(nd_box *b, double *E)
{
    return guarded([&] {
        check_box(b);
        require(E != nullptr, ND_E_INVALID, "E is NULL");
        DeviceGuard g(b->device);
        ND_HIP(hipMemcpyAsync(E, b->E, sizeof(double), hipMemcpyDeviceToHost, b->stream));
        ND_HIP(hipStreamSynchronize(b->stream));
    });
}

nd_status nd_mc_sweep(nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t first_trial,
                      int64_t n_trials, nd_mc_stats *stats, const nd_mc_trace *trace)
{
    return guarded([&] {
        check_box(b);
        require(n_trials >= 0, ND_E_INVALID, "n_trials must be >= 0");
        check_mc_params(b, p);
        DeviceGuard g(b->device);
        // the running energy is brought up to date first when coordinates or
        // tables changed since it was last computed
        if (!b->energy_valid) {
            // O(N) from cell lists (the explicit nd_box_total_energy sums all pairs)
            nd::launch_energy_cells(b, b->E);
            nd::launch_intra_energy_add(b, b->E, nullptr);
            b->energy_valid = true;
        }
        if (b->track.on && !b->track.valid) nd::track_refresh(b);
        nd::mc_run(b, p, seed, first_trial, n_trials, trace);
        if (stats) {
            long long c[2];
            double s;
            ND_HIP(hipMemcpyAsync(c, b->mc.counters, sizeof(c), hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipMemcpyAsync(&s, b->mc.dsum, sizeof(double), hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipMemcpyAsync(&stats->E_total, b->E, sizeof(double), hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
            stats->trials = n_trials;
            stats->accepted = c[0];
            stats->near_ties = c[1];
            stats->dE_sum = s;
        }
    });
}

nd_status nd_pair_histogram(nd_box *b, double dr, int32_t nbins, uint64_t *counts, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(counts != nullptr, ND_E_INVALID, "counts is NULL");
        check_where(where);
        check_hist_range(b, dr, nbins);
        DeviceGuard g(b->device);
        size_t bytes = sizeof(uint64_t) * (size_t)b->P * nbins;
        if (where == ND_DEVICE) {
            nd::launch_pair_histogram(b, dr, nbins, counts);
        } else {
            Scratch s(bytes, b->stream);
            nd::launch_pair_histogram(b, dr, nbins, s.as<uint64_t>());
            ND_HIP(hipMemcpyAsync(counts, s.p, bytes, hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
        }
    });
}

nd_status nd_gr_normalize(const uint64_t *counts, int32_t P, int32_t nbins, double dr, double V,
                          const double *npairs, double *g, int32_t where, void *stream)
{
    return guarded([&] {
        require(counts && npairs && g, ND_E_INVALID, "NULL argument");
        check_where(where);
        require(P >= 1 && P <= ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2, ND_E_INVALID, "P out of range");
        require(nbins >= 1, ND_E_INVALID, "nbins must be >= 1");
        require(std::isfinite(dr) && dr > 0.0 && std::isfinite(V) && V > 0.0, ND_E_INVALID, "dr and V must be > 0");
        for (int p = 0; p < P; ++p)
            require(std::isfinite(npairs[p]) && npairs[p] > 0.0, ND_E_INVALID, "npairs must be > 0");
        hipStream_t s = static_cast<hipStream_t>(stream);
        size_t n = (size_t)P * nbins;
        if (where == ND_DEVICE) {
            nd::launch_gr_normalize(counts, P, nbins, dr, V, npairs, g, s);
        } else {
            Scratch dc(n * sizeof(uint64_t), s), dg(n * sizeof(double), s);
            ND_HIP(hipMemcpyAsync(dc.p, counts, n * sizeof(uint64_t), hipMemcpyHostToDevice, s));
            nd::launch_gr_normalize(dc.as<uint64_t>(), P, nbins, dr, V, npairs, dg.as<double>(), s);
            ND_HIP(hipMemcpyAsync(g, dg.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
            ND_HIP(hipStreamSynchronize(s));
        }
    });
}

nd_status nd_gr_normalize_f64(const double *counts, int32_t P, int32_t nbins, double dr, double V,
                              const double *npairs, double *g, int32_t where, void *stream)
{
    return guarded([&] {
        require(counts && npairs && g, ND_E_INVALID, "NULL argument");
        check_where(where);
        require(P >= 1 && P <= ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2, ND_E_INVALID, "P out of range");
        require(nbins >= 1, ND_E_INVALID, "nbins must be >= 1");
        require(std::isfinite(dr) && dr > 0.0 && std::isfinite(V) && V > 0.0, ND_E_INVALID, "dr and V must be > 0");
        for (int p = 0; p < P; ++p)
            require(std::isfinite(npairs[p]) && npairs[p] > 0.0, ND_E_INVALID, "npairs must be > 0");
        hipStream_t s = static_cast<hipStream_t>(stream);
        size_t n = (size_t)P * nbins;
        if (where == ND_DEVICE) {
            nd::launch_gr_normalize_f64(counts, P, nbins, dr, V, npairs, g, s);
        } else {
            Scratch dc(n * sizeof(double), s), dg(n * sizeof(double), s);
            ND_HIP(hipMemcpyAsync(dc.p, counts, n * sizeof(double), hipMemcpyHostToDevice, s));
            nd::launch_gr_normalize_f64(dc.as<double>(), P, nbins, dr, V, npairs, dg.as<double>(), s);
            ND_HIP(hipMemcpyAsync(g, dg.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
            ND_HIP(hipStreamSynchronize(s));
        }
    });
}

nd_status nd_box_pair_counts(nd_box *b, double *npairs)
{
    return guarded([&] {
        check_box(b);
        require(npairs != nullptr, ND_E_INVALID, "npairs is NULL");
        box_npairs(b, npairs);
    });
}

nd_status nd_box_track_histogram(nd_box *b, double dr, int32_t nbins)
{
    return guarded([&] {
        check_box(b);
        DeviceGuard g(b->device);
        if (nbins == 0) {
            nd::track_stop(b);
            return;
        }
        check_hist_range(b, dr, nbins);
        nd::track_start(b, dr, nbins);
    });
}

nd_status nd_box_tracked_histogram(nd_box *b, uint64_t *counts, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(counts != nullptr, ND_E_INVALID, "counts is NULL");
        check_where(where);
        require(b->track.on, ND_E_STATE, "no histogram is tracked (nd_box_track_histogram)");
        DeviceGuard g(b->device);
        if (!b->track.valid) nd::track_refresh(b);
        const size_t bytes = sizeof(uint64_t) * (size_t)b->P * b->track.nbins;
        if (where == ND_HOST) {
            ND_HIP(hipMemcpyAsync(counts, b->track.counts, bytes, hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
        } else {
            ND_HIP(hipMemcpyAsync(counts, b->track.counts, bytes, hipMemcpyDeviceToDevice, b->stream));
        }
    });
}

nd_status nd_box_accumulate(nd_box *b)
{
    return guarded([&] {
        check_box(b);
        require(b->track.on, ND_E_STATE, "no histogram is tracked (nd_box_track_histogram)");
        DeviceGuard g(b->device);
        if (!b->track.valid) nd::track_refresh(b);
        nd::track_accumulate(b);
    });
}

nd_status nd_box_accumulated(nd_box *b, double *mean_counts, int64_t *n_samples, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(mean_counts != nullptr, ND_E_INVALID, "mean_counts is NULL");
        check_where(where);
        require(b->track.on, ND_E_STATE, "no histogram is tracked (nd_box_track_histogram)");
        require(b->track.n_samples > 0, ND_E_STATE, "no sample accumulated (nd_box_accumulate)");
        DeviceGuard g(b->device);
        const size_t n = (size_t)b->P * b->track.nbins;
        if (where == ND_HOST) {
            Scratch d(n * sizeof(double), b->stream);
            nd::track_mean(b, d.as<double>());
            ND_HIP(hipMemcpyAsync(mean_counts, d.p, n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
        } else {
            nd::track_mean(b, mean_counts);
        }
        if (n_samples) *n_samples = b->track.n_samples;
    });
}

nd_status nd_emp_update(nd_box *b, const nd_emp_params *prm, int32_t n_prof, const double *W,
                        const double *self_terms, const double *g, int32_t nbins, double dr, const double *Q,
                        int32_t nQ, const double *S_exp, double *dS, double *emp, double *C)
{
    return guarded([&] {
        check_box(b);
        require(prm != nullptr && W != nullptr && self_terms != nullptr && g != nullptr && Q != nullptr &&
                    S_exp != nullptr,
                ND_E_INVALID, "NULL argument");
        require(b->has_tables, ND_E_STATE, "nd_box_set_tables has not been called");
        require(n_prof >= 1 && n_prof <= ND_EMP_MAX_PROFILES, ND_E_INVALID, "n_prof must be in 1..ND_EMP_MAX_PROFILES");
        require(prm->n_terms >= 1 && prm->n_terms <= ND_EMP_MAX_TERMS, ND_E_INVALID,
                "n_terms must be in 1..ND_EMP_MAX_TERMS");
        require(std::isfinite(prm->sigma) && prm->sigma > 0.0, ND_E_INVALID, "sigma must be > 0");
        require(std::isfinite(prm->feedback) && prm->feedback > 0.0, ND_E_INVALID, "feedback must be > 0");
        require(std::isfinite(prm->kT) && prm->kT > 0.0, ND_E_INVALID, "kT must be > 0");
        require(std::isfinite(prm->ridge) && prm->ridge >= 0.0, ND_E_INVALID, "ridge must be >= 0");
        require(std::isfinite(prm->id_weight) && prm->id_weight > 0.0, ND_E_INVALID, "id_weight must be > 0");
        require(std::isfinite(prm->emp_max) && prm->emp_max >= 0.0, ND_E_INVALID, "emp_max must be >= 0");
        require(n_prof <= b->P, ND_E_INVALID, "more profiles than pair types");
        require(nbins >= 1 && nQ >= 1 && std::isfinite(dr) && dr > 0.0, ND_E_INVALID, "bad nbins, nQ or dr");
        for (int i = 0; i < n_prof; ++i) {
            require(std::isfinite(self_terms[i]), ND_E_INVALID, "self term is not finite");
            for (int p = 0; p < b->P; ++p)
                require(std::isfinite(W[(size_t)i * b->P + p]), ND_E_INVALID, "weight is not finite");
        }
        if (n_prof == b->P) {
            // a square weight matrix must be invertible: reject a (near) zero pivot
            std::vector<double> A(W, W + (size_t)n_prof * b->P);
            const int P = b->P;
            double scale = 0.0;
            for (double v : A) scale = std::max(scale, std::fabs(v));
            for (int c = 0; c < P; ++c) {
                int piv = c;
                for (int r = c + 1; r < P; ++r)
                    if (std::fabs(A[r * P + c]) > std::fabs(A[piv * P + c])) piv = r;
                require(std::fabs(A[piv * P + c]) > 1e-12 * scale, ND_E_INVALID, "weight matrix is singular");
                for (int k = 0; k < P; ++k) std::swap(A[c * P + k], A[piv * P + k]);
                for (int r = c + 1; r < P; ++r) {
                    const double f = A[r * P + c] / A[c * P + c];
                    for (int k = c; k < P; ++k) A[r * P + k] -= f * A[c * P + k];
                }
            }
        }
        DeviceGuard dg(b->device);
        nd::launch_emp_update(b, prm, n_prof, W, self_terms, g, nbins, dr, Q, nQ, S_exp, dS, emp, C);
        b->energy_valid = false;
    });
}

nd_status nd_box_get_tables(nd_box *b, float *U, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(U != nullptr, ND_E_INVALID, "U is NULL");
        check_where(where);
        require(b->has_tables, ND_E_STATE, "nd_box_set_tables has not been called");
        DeviceGuard g(b->device);
        const size_t bytes = sizeof(float) * (size_t)b->P * b->n_pts;
        if (where == ND_HOST) {
            ND_HIP(hipMemcpyAsync(U, b->tab, bytes, hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
        } else {
            ND_HIP(hipMemcpyAsync(U, b->tab, bytes, hipMemcpyDeviceToDevice, b->stream));
        }
    });
}

nd_status nd_box_density(nd_box *b, double *V, double *rho)
{
    return guarded([&] {
        check_box(b);
        require(V != nullptr && rho != nullptr, ND_E_INVALID, "NULL argument");
        *V = b->L * b->L * b->L;
        *rho = (double)b->N / *V;
    });
}

nd_status nd_eq1_weights(nd_box *b, const double *bl, double *w, double *self_term)
{
    return guarded([&] {
        check_box(b);
        require(bl && w && self_term, ND_E_INVALID, "NULL argument");
        for (int a = 0; a < b->M; ++a) require(std::isfinite(bl[a]), ND_E_INVALID, "b is not finite");
        double flat = 0.0;
        for (int a = 0; a < b->M; ++a) {
            const double ca = (double)b->species_count[a] / (double)b->N;
            flat += ca * bl[a] * bl[a];
            for (int c = a; c < b->M; ++c) {
                const double cc = (double)b->species_count[c] / (double)b->N;
                w[nd::pair_index(a, c, b->M)] = (a == c ? 1.0 : 2.0) * ca * cc * bl[a] * bl[c];
            }
        }
        *self_term = flat;
    });
}

nd_status nd_chi2(const double *S, const double *T, int32_t nQ, double *chi2, double *grad, int32_t where,
                  void *stream)
{
    return guarded([&] {
        require(S && T && chi2, ND_E_INVALID, "NULL argument");
        check_where(where);
        require(nQ >= 1, ND_E_INVALID, "nQ must be >= 1");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (where == ND_DEVICE) {
            nd::launch_chi2(S, T, nQ, chi2, grad, s);
        } else {
            size_t n = (size_t)nQ * sizeof(double);
            Scratch ds(n, s), dt(n, s), dg(n, s), dc(sizeof(double), s);
            ND_HIP(hipMemcpyAsync(ds.p, S, n, hipMemcpyHostToDevice, s));
            ND_HIP(hipMemcpyAsync(dt.p, T, n, hipMemcpyHostToDevice, s));
            nd::launch_chi2(ds.as<double>(), dt.as<double>(), nQ, dc.as<double>(), dg.as<double>(), s);
            ND_HIP(hipMemcpyAsync(chi2, dc.p, sizeof(double), hipMemcpyDeviceToHost, s));
            if (grad) ND_HIP(hipMemcpyAsync(grad, dg.p, n, hipMemcpyDeviceToHost, s));
            ND_HIP(hipStreamSynchronize(s));
        }
    });
}

nd_status nd_sq_transform(const double *g, int32_t P, int32_t nbins, double dr, double rho,
                          const double *w, double self_term, const double *Q, int32_t nQ,
                          double *S, int32_t where, void *stream)
{
    return guarded([&] {
        require(g && w && Q && S, ND_E_INVALID, "NULL argument");
        check_where(where);
        require(P >= 1 && P <= ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2, ND_E_INVALID, "P out of range");
        require(nbins >= 1 && nQ >= 1, ND_E_INVALID, "nbins and nQ must be >= 1");
        require(std::isfinite(dr) && dr > 0.0, ND_E_INVALID, "dr must be > 0");
        require(std::isfinite(rho) && rho > 0.0 && std::isfinite(self_term), ND_E_INVALID, "bad rho or self_term");
        for (int p = 0; p < P; ++p) require(std::isfinite(w[p]), ND_E_INVALID, "weight is not finite");
        hipStream_t s = static_cast<hipStream_t>(stream);
        size_t n = (size_t)P * nbins;
        if (where == ND_DEVICE) {
            nd::launch_sq(g, P, nbins, dr, rho, w, self_term, Q, nQ, S, s);
        } else {
            Scratch dg(n * sizeof(double), s), dq(nQ * sizeof(double), s), ds(nQ * sizeof(double), s);
            ND_HIP(hipMemcpyAsync(dg.p, g, n * sizeof(double), hipMemcpyHostToDevice, s));
            ND_HIP(hipMemcpyAsync(dq.p, Q, nQ * sizeof(double), hipMemcpyHostToDevice, s));
            nd::launch_sq(dg.as<double>(), P, nbins, dr, rho, w, self_term, dq.as<double>(), nQ, ds.as<double>(), s);
            ND_HIP(hipMemcpyAsync(S, ds.p, nQ * sizeof(double), hipMemcpyDeviceToHost, s));
            ND_HIP(hipStreamSynchronize(s));
        }
    });
}

nd_status nd_hist_broad(nd_box *b, double dr, int32_t nbins, double sigma, double *nhat, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(nhat != nullptr, ND_E_INVALID, "nhat is NULL");
        check_where(where);
        require(std::isfinite(dr) && dr > 0.0 && nbins >= 1, ND_E_INVALID, "bad dr or nbins");
        require(std::isfinite(sigma) && sigma > 0.0, ND_E_INVALID, "sigma must be > 0");
        require(6.0 * sigma < 8.0 * dr, ND_E_UNSUPPORTED, "6 sigma must be < 8 dr");
        require((double)nbins * dr < 0.5 * b->L * (1.0 - 1e-9), ND_E_RANGE, "nbins*dr must be < L/2");
        DeviceGuard g(b->device);
        size_t bytes = sizeof(double) * (size_t)b->P * nbins;
        if (where == ND_DEVICE) {
            nd::launch_hist_broad(b, dr, nbins, sigma, nhat);
        } else {
            Scratch s(bytes, b->stream);
            nd::launch_hist_broad(b, dr, nbins, sigma, s.as<double>());
            ND_HIP(hipMemcpyAsync(nhat, s.p, bytes, hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
        }
    });
}

nd_status nd_sq_adjoint(const double *dLdS, int32_t P, int32_t nbins, double dr, double rho, double V,
                        const double *w, const double *npairs, const double *Q, int32_t nQ, double *A,
                        int32_t where, void *stream)
{
    return guarded([&] {
        require(dLdS && w && npairs && Q && A, ND_E_INVALID, "NULL argument");
        check_where(where);
        require(P >= 1 && P <= ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2, ND_E_INVALID, "P out of range");
        require(nbins >= 1 && nQ >= 1, ND_E_INVALID, "nbins and nQ must be >= 1");
        require(std::isfinite(dr) && dr > 0.0 && std::isfinite(rho) && rho > 0.0 && std::isfinite(V) && V > 0.0,
                ND_E_INVALID, "dr, rho and V must be > 0");
        for (int p = 0; p < P; ++p)
            require(std::isfinite(w[p]) && std::isfinite(npairs[p]) && npairs[p] > 0.0, ND_E_INVALID,
                    "bad weight or npairs");
        hipStream_t s = static_cast<hipStream_t>(stream);
        size_t n = (size_t)P * nbins;
        if (where == ND_DEVICE) {
            nd::launch_sq_adjoint(dLdS, P, nbins, dr, rho, V, w, npairs, Q, nQ, A, s);
        } else {
            Scratch dd(nQ * sizeof(double), s), dq(nQ * sizeof(double), s), da(n * sizeof(double), s);
            ND_HIP(hipMemcpyAsync(dd.p, dLdS, nQ * sizeof(double), hipMemcpyHostToDevice, s));
            ND_HIP(hipMemcpyAsync(dq.p, Q, nQ * sizeof(double), hipMemcpyHostToDevice, s));
            nd::launch_sq_adjoint(dd.as<double>(), P, nbins, dr, rho, V, w, npairs, dq.as<double>(), nQ,
                                  da.as<double>(), s);
            ND_HIP(hipMemcpyAsync(A, da.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
            ND_HIP(hipStreamSynchronize(s));
        }
    });
}

nd_status nd_hist_broad_backward(nd_box *b, double dr, int32_t nbins, double sigma, const double *A,
                                 double *dLdx, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(A != nullptr && dLdx != nullptr, ND_E_INVALID, "NULL argument");
        check_where(where);
        require(std::isfinite(dr) && dr > 0.0 && nbins >= 1, ND_E_INVALID, "bad dr or nbins");
        require(std::isfinite(sigma) && sigma > 0.0, ND_E_INVALID, "sigma must be > 0");
        require(6.0 * sigma < 8.0 * dr, ND_E_UNSUPPORTED, "6 sigma must be < 8 dr");
        require((double)nbins * dr < 0.5 * b->L * (1.0 - 1e-9), ND_E_RANGE, "nbins*dr must be < L/2");
        DeviceGuard g(b->device);
        size_t nA = (size_t)b->P * nbins, nG = (size_t)3 * b->N;
        if (where == ND_DEVICE) {
            nd::launch_hist_broad_backward(b, dr, nbins, sigma, A, dLdx);
        } else {
            Scratch da(nA * sizeof(double), b->stream), dg(nG * sizeof(double), b->stream);
            ND_HIP(hipMemcpyAsync(da.p, A, nA * sizeof(double), hipMemcpyHostToDevice, b->stream));
            nd::launch_hist_broad_backward(b, dr, nbins, sigma, da.as<double>(), dg.as<double>());
            ND_HIP(hipMemcpyAsync(dLdx, dg.p, nG * sizeof(double), hipMemcpyDeviceToHost, b->stream));
            ND_HIP(hipStreamSynchronize(b->stream));
        }
    });
}

nd_status nd_forces(nd_box *b, double *dEdx, double *E, int32_t where)
{
    return guarded([&] {
        check_box(b);
        require(dEdx != nullptr, ND_E_INVALID, "dEdx is NULL");
        check_where(where);
        require(b->has_tables, ND_E_STATE, "nd_box_set_tables has not been called");
        DeviceGuard g(b->device);
        size_t nG = (size_t)3 * b->N;
        Scratch de(sizeof(double), b->stream);
        if (where == ND_DEVICE) {
            nd::launch_forces(b, dEdx, de.as<double>());
        } else {
            Scratch dg(nG * sizeof(double), b->stream);
            nd::launch_forces(b, dg.as<double>(), de.as<double>());
            ND_HIP(hipMemcpyAsync(dEdx, dg.p, nG * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        }
        if (E) {
            ND_HIP(hipMemcpyAsync(E, de.p, sizeof(double), hipMemcpyDeviceToHost, b->stream));
        }
        ND_HIP(hipStreamSynchronize(b->stream));
    });
}

namespace {
std::mutex g_scratch_mu;
char *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on `device` (current), looked up once per device.
char *noalloc_scratch(int device)
{
    require(device >= 0 && device < NOALLOC_MAX_DEVICES, ND_E_UNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        ND_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        require(ptr != nullptr, ND_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_dev[device] = static_cast<char *>(ptr);
    }
    return g_scratch_dev[device];
}
}  // namespace

nd_status nd_forces_noalloc(nd_box *b, double *dEdx, double *E)
{
    return guarded([&] {
        check_box(b);
        require(dEdx != nullptr, ND_E_INVALID, "dEdx is NULL");
        require(b->has_tables, ND_E_STATE, "nd_box_set_tables has not been called");
        require(b->N <= ND_NOALLOC_MAX_ATOMS, ND_E_RANGE,
                "nd_forces_noalloc takes at most ND_NOALLOC_MAX_ATOMS (262144) atoms");
        DeviceGuard g(b->device);
        char *ws = noalloc_scratch(b->device);
        double *e_out = E ? E : reinterpret_cast<double *>(ws + NOALLOC_FORCES_BYTES);
        nd::launch_forces_in(b, dEdx, e_out, ws, NOALLOC_MAX_GRID, false);
    });
}

nd_status nd_set_tuning(const nd_tuning *entries, int32_t n)
{
    return guarded([&] {
        require(n >= 0 && (n == 0 || entries != nullptr), ND_E_INVALID, "entries is NULL or n < 0");
        for (int i = 0; i < n; ++i) check_tuning(entries[i]);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.assign(entries, entries + n);
    });
}

nd_status nd_get_tuning(nd_tuning *entries, int32_t cap, int32_t *n)
{
    return guarded([&] {
        require(n != nullptr && cap >= 0 && (cap == 0 || entries != nullptr), ND_E_INVALID, "bad arguments");
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int i = 0; i < cap && i < (int)g_tune.size(); ++i) entries[i] = g_tune[i];
        *n = (int32_t)g_tune.size();
    });
}

nd_status nd_load_tuning(const char *path)
{
    return guarded([&] {
        require(path != nullptr, ND_E_INVALID, "path is NULL");
        FILE *f = std::fopen(path, "r");
        require(f != nullptr, ND_E_INVALID, std::string("cannot open ") + path);
        std::vector<nd_tuning> t;
        char line[512];
        int lineno = 0;
        bool ok = true;
        std::string bad;
        while (std::fgets(line, sizeof(line), f)) {
            ++lineno;
            char *q = line;
            while (*q == ' ' || *q == '\t') ++q;
            if (*q == '#' || *q == '\n' || *q == '\r' || *q == 0) continue;
            char kind[16];
            long long n_max = 0;
            int waves = 0, bpc = 0;
            double target = 0.0;
            if (std::sscanf(q, "%15s %lld %d %lf %d", kind, &n_max, &waves, &target, &bpc) != 5) {
                ok = false;
                bad = "malformed line " + std::to_string(lineno);
                break;
            }
            nd_tuning e;
            std::memset(&e, 0, sizeof(e));
            e.kind = std::strcmp(kind, "box") == 0 ? ND_TUNE_BOX : (std::strcmp(kind, "batch") == 0 ? ND_TUNE_BATCH : -1);
            e.n_max = n_max;
            e.scan_waves = waves;
            e.batch_target = target;
            e.hist_blocks_per_cu = bpc;
            t.push_back(e);
        }
        std::fclose(f);
        require(ok, ND_E_INVALID, std::string(path) + ": " + bad);
        for (const nd_tuning &e : t) check_tuning(e);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune = t;
    });
}

nd_status nd_batch_create(nd_box *const *boxes, int32_t n, nd_batch **out)
{
    return guarded([&] {
        require(out != nullptr, ND_E_INVALID, "out is NULL");
        *out = nullptr;
        require(boxes != nullptr && n >= 1, ND_E_INVALID, "boxes is NULL or n < 1");
        for (int i = 0; i < n; ++i) {
            check_box(boxes[i]);
            require(boxes[i]->device == boxes[0]->device, ND_E_INVALID, "boxes are on different devices");
            require(boxes[i]->M == boxes[0]->M, ND_E_INVALID, "boxes have different species counts");
            for (int j = 0; j < i; ++j) require(boxes[j] != boxes[i], ND_E_INVALID, "a box appears twice");
        }
        DeviceGuard g(boxes[0]->device);
        nd_batch *t = new nd_batch();
        try {
            t->boxes.assign(boxes, boxes + n);
            t->device = boxes[0]->device;
            ND_HIP(hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking));
            ND_HIP(hipEventCreateWithFlags(&t->ev_done, hipEventDisableTiming));
            t->ev_in.resize(n, nullptr);
            for (int i = 0; i < n; ++i) ND_HIP(hipEventCreateWithFlags(&t->ev_in[i], hipEventDisableTiming));
            t->mc = nd::mc_multi_create();
            t->hist = nd::hist_multi_create();
            t->sq = nd::sq_multi_create();
        } catch (...) {
            free_batch(t);
            throw;
        }
        *out = t;
    });
}

nd_status nd_batch_destroy(nd_batch *t)
{
    if (!t) return ND_OK;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(t->device) != hipSuccess) {
        // runtime no longer usable (process teardown): host side only
        (void)hipGetLastError();
        delete t;
        return ND_OK;
    }
    free_batch(t);
    if (prev >= 0) (void)hipSetDevice(prev);
    return ND_OK;
}

nd_status nd_batch_run(nd_batch *t, const nd_batch_plan *pl, nd_mc_stats *stats)
{
    return guarded([&] {
        require(t != nullptr, ND_E_INVALID, "batch is NULL");
        require(pl != nullptr, ND_E_INVALID, "plan is NULL");
        const int n = (int)t->boxes.size();
        nd_box *const *boxes = t->boxes.data();
        // ---- validation, before any device work
        require(pl->sweeps >= 0, ND_E_INVALID, "sweeps must be >= 0");
        if (pl->sweeps > 0) {
            require(pl->mc && pl->seed && pl->first_trial, ND_E_INVALID, "mc, seed and first_trial are required");
            for (int i = 0; i < n; ++i) {
                check_mc_params(boxes[i], &pl->mc[i]);
                require(pl->mc[i].scan == ND_SCAN_CELLS, ND_E_UNSUPPORTED, "the batched form runs the cell scan only");
            }
        }
        const bool do_hist = pl->counts != nullptr;
        const bool do_g = do_hist && pl->g != nullptr;
        const bool do_s = do_g && pl->S != nullptr && pl->nQ > 0;
        if (do_hist) {
            require(pl->nbins != nullptr, ND_E_INVALID, "nbins is NULL");
            for (int i = 0; i < n; ++i) {
                check_hist_range(boxes[i], pl->dr, pl->nbins[i]);
                require(pl->counts[i] != nullptr, ND_E_INVALID, "counts[i] is NULL");
                if (do_g) require(pl->g[i] != nullptr, ND_E_INVALID, "g[i] is NULL");
            }
        }
        if (do_s) {
            require(pl->Q && pl->w && pl->self_term, ND_E_INVALID, "Q, w and self_term are required for S");
            for (int i = 0; i < n; ++i) {
                require(pl->S[i] != nullptr, ND_E_INVALID, "S[i] is NULL");
                require(std::isfinite(pl->self_term[i]), ND_E_INVALID, "self_term is not finite");
                for (int p = 0; p < boxes[i]->P; ++p)
                    require(std::isfinite(pl->w[(size_t)i * boxes[i]->P + p]), ND_E_INVALID, "w is not finite");
            }
        }
        DeviceGuard g(t->device);
        hipStream_t s = t->stream;
        // the previous run has finished reading the descriptors
        ND_HIP(hipStreamSynchronize(s));
        // ---- host plan and descriptor upload
        std::vector<long long> sig;
        if (pl->sweeps > 0) {
            std::vector<int64_t> nt(n);
            for (int i = 0; i < n; ++i) nt[i] = (int64_t)pl->sweeps * boxes[i]->n_units;
            nd::mc_multi_plan(t->mc, boxes, n, pl->mc, pl->seed, pl->first_trial, nt.data(), pl->trace, sig);
            nd::mc_multi_upload(t->mc, s);
        }
        sig.push_back(-1);
        if (do_hist) {
            nd::hist_multi_plan(t->hist, boxes, n, pl->dr, pl->nbins, pl->counts, sig);
            nd::hist_multi_upload(t->hist, s);
        }
        sig.push_back(-2);
        if (do_g) {
            std::vector<nd::SqBoxDesc> d(n);
            for (int i = 0; i < n; ++i) {
                const nd_box *b = boxes[i];
                nd::SqBoxDesc &x = d[i];
                std::memset(&x, 0, sizeof(x));
                x.counts = pl->counts[i];
                x.g = pl->g[i];
                x.S = do_s ? pl->S[i] : nullptr;
                x.P = b->P;
                x.nbins = pl->nbins[i];
                x.dr = pl->dr;
                x.V = b->L * b->L * b->L;
                x.four_pi_rho = 4.0 * M_PI * ((double)b->N / x.V);
                x.self_term = do_s ? pl->self_term[i] : 0.0;
                box_npairs(b, x.npairs);
                if (do_s)
                    for (int p = 0; p < b->P; ++p) x.w[p] = pl->w[(size_t)i * b->P + p];
            }
            nd::sq_multi_plan(t->sq, d.data(), n, do_s ? pl->Q : nullptr, do_s ? pl->nQ : 0, sig);
            nd::sq_multi_upload(t->sq, s);
        }
        // running energies brought up to date on the boxes' own streams
        if (pl->sweeps > 0)
            for (int i = 0; i < n; ++i)
                if (!boxes[i]->energy_valid) {
                    nd::launch_energy_cells(boxes[i], boxes[i]->E);
                    nd::launch_intra_energy_add(boxes[i], boxes[i]->E, nullptr);
                    boxes[i]->energy_valid = true;
                }
        // ---- order after pending work on the boxes' streams
        for (int i = 0; i < n; ++i) {
            ND_HIP(hipEventRecord(t->ev_in[i], boxes[i]->stream));
            ND_HIP(hipStreamWaitEvent(s, t->ev_in[i], 0));
        }
        // ---- capture once per launch structure, then replay
        if (!t->exec || sig != t->sig) {
            if (t->exec) {
                ND_HIP(hipGraphExecDestroy(t->exec));
                t->exec = nullptr;
            }
            if (t->graph) {
                ND_HIP(hipGraphDestroy(t->graph));
                t->graph = nullptr;
            }
            t->sig.clear();
            ND_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                if (pl->sweeps > 0) nd::mc_multi_enqueue(t->mc, s);
                if (do_hist) nd::hist_multi_enqueue(t->hist, s);
                if (do_g) nd::sq_multi_enqueue(t->sq, s);
            } catch (...) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(s, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                throw;
            }
            ND_HIP(hipStreamEndCapture(s, &t->graph));
            ND_HIP(hipGraphInstantiate(&t->exec, t->graph, nullptr, nullptr, 0));
            t->sig = sig;
            ++t->captures;
        }
        ND_HIP(hipGraphLaunch(t->exec, s));
        ++t->launches;
        // the batched sweeps do not update running histograms
        if (pl->sweeps > 0)
            for (int i = 0; i < n; ++i) boxes[i]->track.valid = false;
        // later work on the boxes' streams comes after the batch
        ND_HIP(hipEventRecord(t->ev_done, s));
        for (int i = 0; i < n; ++i) ND_HIP(hipStreamWaitEvent(boxes[i]->stream, t->ev_done, 0));
        if (stats) {
            ND_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < n; ++i) {
                nd_box *b = boxes[i];
                nd_mc_stats &st = stats[i];
                std::memset(&st, 0, sizeof(st));
                if (pl->sweeps > 0) {
                    long long c[2];
                    ND_HIP(hipMemcpy(c, b->mc.counters, sizeof(c), hipMemcpyDeviceToHost));
                    ND_HIP(hipMemcpy(&st.dE_sum, b->mc.dsum, sizeof(double), hipMemcpyDeviceToHost));
                    st.trials = (int64_t)pl->sweeps * b->n_units;
                    st.accepted = c[0];
                    st.near_ties = c[1];
                }
                ND_HIP(hipMemcpy(&st.E_total, b->E, sizeof(double), hipMemcpyDeviceToHost));
            }
        }
    });
}

nd_status nd_batch_info(const nd_batch *t, int64_t *captures, int64_t *launches)
{
    return guarded([&] {
        require(t != nullptr, ND_E_INVALID, "batch is NULL");
        if (captures) *captures = t->captures;
        if (launches) *launches = t->launches;
    });
}

nd_status nd_box_save(nd_box *b, void *buf, size_t *len)
{
    return guarded([&] {
        check_box(b);
        require(len != nullptr, ND_E_INVALID, "len is NULL");
        const bool cells = b->cells.valid;
        const size_t need = ckpt_size(b, cells, b->cells.ncell);
        if (buf == nullptr) {
            *len = need;
            return;
        }
        require(*len >= need, ND_E_INVALID, "buffer too small for the checkpoint");
        DeviceGuard g(b->device);
        ND_HIP(hipStreamSynchronize(b->stream));
        unsigned char *p = static_cast<unsigned char *>(buf);
        CkptHeader h;
        std::memset(&h, 0, sizeof(h));
        std::memcpy(h.magic, CKPT_MAGIC, 8);
        h.version = 1;
        h.n_atoms = b->N;
        h.n_species = b->M;
        h.n_units = b->n_units;
        h.L = b->L;
        ND_HIP(hipMemcpy(&h.E, b->E, sizeof(double), hipMemcpyDeviceToHost));
        h.energy_valid = b->energy_valid ? 1 : 0;
        h.cells_valid = cells ? 1 : 0;
        h.nc = cells ? b->cells.nc : 0;
        h.ncell = cells ? b->cells.ncell : 0;
        h.trials_since_build = cells ? b->cells.trials_since_build : 0;
        if (cells) ND_HIP(hipMemcpy(&h.drift, b->cells.drift, sizeof(float), hipMemcpyDeviceToHost));
        std::memcpy(p, &h, sizeof(h));
        size_t off = sizeof(h);
        const size_t N = (size_t)b->N;
        ND_HIP(hipMemcpy(p + off, b->xyz, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
        off += sizeof(float) * 3 * N;
        if (cells) {
            const nd::Cells &c = b->cells;
            ND_HIP(hipMemcpy(p + off, c.sorted, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
            off += sizeof(int32_t) * N;
            ND_HIP(hipMemcpy(p + off, c.slot, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
            off += sizeof(int32_t) * N;
            ND_HIP(hipMemcpy(p + off, c.start, sizeof(int32_t) * (c.ncell + 1), hipMemcpyDeviceToHost));
            off += sizeof(int32_t) * (c.ncell + 1);
            ND_HIP(hipMemcpy(p + off, c.sref, sizeof(float4) * N, hipMemcpyDeviceToHost));
            off += sizeof(float4) * N;
        }
        const uint64_t hash = fnv1a(p, off);
        std::memcpy(p + off, &hash, sizeof(hash));
        *len = off + sizeof(hash);
    });
}

nd_status nd_box_load(nd_box *b, const void *buf, size_t len)
{
    return guarded([&] {
        check_box(b);
        require(buf != nullptr, ND_E_INVALID, "buffer is NULL");
        const unsigned char *p = static_cast<const unsigned char *>(buf);
        require(len >= sizeof(CkptHeader) + sizeof(uint64_t), ND_E_INVALID, "checkpoint truncated");
        CkptHeader h;
        std::memcpy(&h, p, sizeof(h));
        require(std::memcmp(h.magic, CKPT_MAGIC, 8) == 0 && h.version == 1, ND_E_INVALID, "not a box checkpoint");
        require(h.n_atoms == b->N && h.n_species == b->M && h.n_units == b->n_units && h.L == b->L,
                ND_E_INVALID, "checkpoint is of a different box");
        const bool cells = h.cells_valid != 0;
        require(!cells || (h.ncell == h.nc * h.nc * h.nc && h.nc >= 1), ND_E_INVALID, "bad cell grid");
        const size_t need = ckpt_size(b, cells, h.ncell);
        require(len >= need, ND_E_INVALID, "checkpoint truncated");
        uint64_t hash;
        std::memcpy(&hash, p + need - sizeof(hash), sizeof(hash));
        require(hash == fnv1a(p, need - sizeof(hash)), ND_E_INVALID, "checkpoint hash mismatch");
        const size_t N = (size_t)b->N;
        const float *xyz = reinterpret_cast<const float *>(p + sizeof(h));
        validate_xyz_host(xyz, b->N, b->L);
        DeviceGuard g(b->device);
        ND_HIP(hipStreamSynchronize(b->stream));
        ND_HIP(hipMemcpy(b->xyz, xyz, sizeof(float) * 3 * N, hipMemcpyHostToDevice));
        nd::launch_pos4_from_xyz(b);
        ND_HIP(hipMemcpyAsync(b->E, &h.E, sizeof(double), hipMemcpyHostToDevice, b->stream));
        ND_HIP(hipStreamSynchronize(b->stream));
        b->energy_valid = h.energy_valid != 0;
        b->cells.valid = false;
        b->track.valid = false;
        if (cells) {
            size_t off = sizeof(h) + sizeof(float) * 3 * N;
            nd::CellState st;
            st.nc = h.nc;
            st.trials_since_build = h.trials_since_build;
            st.drift = h.drift;
            st.sorted = reinterpret_cast<const int32_t *>(p + off);
            off += sizeof(int32_t) * N;
            st.slot = reinterpret_cast<const int32_t *>(p + off);
            off += sizeof(int32_t) * N;
            st.start = reinterpret_cast<const int32_t *>(p + off);
            off += sizeof(int32_t) * (h.ncell + 1);
            st.sref = reinterpret_cast<const float4 *>(p + off);
            // a permutation with matching inverse, and a monotone start table
            std::vector<char> seen(N, 0);
            for (size_t x = 0; x < N; ++x) {
                const int32_t a = st.sorted[x];
                require(a >= 0 && (size_t)a < N && !seen[a] && st.slot[a] == (int32_t)x, ND_E_INVALID,
                        "checkpoint cell order is corrupt");
                seen[a] = 1;
            }
            require(st.start[0] == 0 && st.start[h.ncell] == b->N, ND_E_INVALID, "checkpoint cell table is corrupt");
            for (int c = 0; c < h.ncell; ++c)
                require(st.start[c] <= st.start[c + 1], ND_E_INVALID, "checkpoint cell table is corrupt");
            nd::cells_restore(b, st);
        }
    });
}

}  // extern "C"
