// pflbm_runtime.hip -- host runtime behind the C ABI of include/pflbm.h.
//
// Validates parameters, carves the caller's workspace into per-case state
// planes, builds the tile table of the batched launch and enqueues kernels on
// the caller's stream.  The library never allocates device memory.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "pflbm.h"
#include "pflbm_internal.h"

using namespace pflbm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kPitchElems = 64;
constexpr int kReduceMax = 1024;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Scratch of pflbm_bubble_centroid_velocity_noalloc: the reduction partials
// of at most kReduceMax blocks (6 float64 each) followed by the 6 final sums
// (8 slots).  One copy per GPU, held until the process ends; host code uses
// the address resolved per device below, never the symbol itself.
constexpr size_t kScratchDoubles = 6 * (size_t)kReduceMax + 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, resolved once per device with
// that device current (the caller's current device at pflbm_create).
hipError_t scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

struct CaseLayout {
    size_t P[2], S[2], C[2], T[2], H[2], Q[2];   // byte offsets into the workspace; P[b] starts buffer b
    int pitch;
    long long plane;                 // elements per plane
};

struct Layout {
    size_t cases_off, tiles_off, result_off, partial_off, flags_off, staging_off;
    size_t staging_bytes;
    size_t max_tiles;
    std::vector<CaseLayout> cl;
    size_t state_begin, state_end;   // byte range of all state planes
    size_t total;
};

// Capillary coefficients Sigma_i = sigma_ij + sigma_ik - sigma_jk and Sigma_T (Sec. 2.1).
void capillary(const pflbm_params& p, double S[3], double* ST) {
    S[0] = p.sigma12 + p.sigma13 - p.sigma23;
    S[1] = p.sigma12 + p.sigma23 - p.sigma13;
    S[2] = p.sigma13 + p.sigma23 - p.sigma12;
    *ST = 3.0 / (1.0 / S[0] + 1.0 / S[1] + 1.0 / S[2]);
}

bool is_finite(double v) { return isfinite(v) != 0; }

bool valid_params(const pflbm_params& p) {
    if (p.nx < 5 || p.ny < 5 || (p.n_h != 1 && p.n_h != 2)) return false;
    // kernels address a plane with 32-bit byte offsets: float64 planes < 4 GiB
    if ((double)align_up((size_t)p.nx, kPitchElems) * (double)p.ny * 8.0 >= 4294967296.0) return false;
    if ((long long)p.nx * p.ny > (1LL << 31)) return false;
    for (int k = 0; k < 3; ++k)
        if (!(p.rho[k] > 0.0) || !(p.nu[k] > 0.0) || !is_finite(p.rho[k]) || !is_finite(p.nu[k])) return false;
    if (p.powerlaw_comp < -1 || p.powerlaw_comp > 2) return false;
    if (p.powerlaw_comp >= 0) {
        if (!(p.K > 0.0) || !is_finite(p.K) || !(p.n > 0.0) || !is_finite(p.n) || !(p.nu_min > 0.0) ||
            !(p.nu_min <= p.nu_max) || !is_finite(p.nu_max))
            return false;
    }
    if (!(p.xi > 0.0) || !(p.D0 >= 0.0) || !(p.tau_h > 0.0)) return false;
    if (!is_finite(p.xi) || !is_finite(p.D0) || !is_finite(p.tau_h)) return false;
    if (!is_finite(p.g) || !is_finite(p.fx) || !is_finite(p.Lambda)) return false;
    double S[3], ST;
    capillary(p, S, &ST);
    for (int k = 0; k < 3; ++k)
        if (!(S[k] > 0.0) || !is_finite(S[k])) return false;
    if (p.storage != 0 && p.storage != 1) return false;
    if (p.store_h != 0 && p.store_h != 1) return false;
    if (!p.store_h && p.tau_h != 0.5) return false;
    if (p.tau_iterations < 0 || p.tau_iterations > 8) return false;
    if (p.hforce_cd != 0 && p.hforce_cd != 1) return false;
    if (p.open_x != 0 && p.open_x != 1) return false;
    if (p.open_x && !is_finite(p.u_in)) return false;
    if (p.mobility_flux != 0 && p.mobility_flux != 1) return false;
    return true;
}

size_t max_tiles_for(const pflbm_params* cases, int n) {
    size_t worst = 0;
    for (int v = 0; v < step_variant_count(); ++v) {
        int tx, ty, nt;
        if (!step_variant_shape(v, cases[0].n_h, &tx, &ty, &nt)) continue;
        size_t t = 0;
        for (int c = 0; c < n; ++c) t += (size_t)((cases[c].nx + tx - 1) / tx) * ((cases[c].ny + ty - 1) / ty);
        if (t > worst) worst = t;
    }
    return worst;
}

bool make_layout(const pflbm_params* cases, int n, Layout* L) {
    if (!cases || n <= 0) return false;
    for (int c = 0; c < n; ++c) {
        if (!valid_params(cases[c])) return false;
        if (cases[c].n_h != cases[0].n_h || cases[c].storage != cases[0].storage ||
            cases[c].store_h != cases[0].store_h)
            return false;
    }
    size_t off = 0;
    L->cases_off = off;
    off = align_up(off + sizeof(CaseDev) * n, kAlign);
    L->max_tiles = max_tiles_for(cases, n);
    L->tiles_off = off;
    off = align_up(off + sizeof(TileDev) * L->max_tiles, kAlign);
    L->result_off = off;
    off = align_up(off + 8 * sizeof(double), kAlign);
    L->partial_off = off;
    off = align_up(off + 6 * sizeof(double) * kReduceMax, kAlign);
    L->flags_off = off;                                  // one non-finite flag per case
    off = align_up(off + sizeof(unsigned int) * n, kAlign);
    size_t maxcells = 0;
    for (int c = 0; c < n; ++c) {
        size_t cells = (size_t)cases[c].nx * cases[c].ny;
        if (cells > maxcells) maxcells = cells;
    }
    L->staging_off = off;
    L->staging_bytes = sizeof(double) * maxcells * (size_t)(cases[0].n_h + 3);
    off = align_up(off + L->staging_bytes, kAlign);
    L->state_begin = off;
    L->cl.resize(n);
    for (int c = 0; c < n; ++c) {
        const pflbm_params& p = cases[c];
        CaseLayout& cl = L->cl[c];
        cl.pitch = (int)align_up((size_t)p.nx, kPitchElems);
        cl.plane = (long long)cl.pitch * p.ny;
        const size_t pb = sizeof(float) * (size_t)cl.plane;
        const bool f16 = p.storage == 1;
        for (int b = 0; b < 2; ++b) {
            cl.P[b] = off; off = align_up(off + 2 * pb, kAlign);                      // float64
            cl.S[b] = off; off = align_up(off + (f16 ? kSPlanes16 : 8) * pb, kAlign);
            if (f16) { cl.Q[b] = off; off = align_up(off + kQPlanes * (pb / 2), kAlign); }
            else cl.Q[b] = 0;
            cl.C[b] = off; off = align_up(off + (size_t)p.n_h * 2 * pb, kAlign);   // float64
            cl.T[b] = off; off = align_up(off + pb, kAlign);
            if (p.store_h) { cl.H[b] = off; off = align_up(off + 9 * (size_t)p.n_h * pb, kAlign); }
            else cl.H[b] = 0;
        }
    }
    L->state_end = off;
    L->total = off;
    return true;
}

}  // namespace

struct pflbm_ctx {
    std::vector<pflbm_params> prm;
    std::vector<CaseDev> cd;          // host copies of the device case blocks
    std::vector<int> initialised;
    std::vector<int> nonfinite;       // sticky: a synchronising call saw the case's flag set
    Layout L;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    int par = 0;
    int variant = 0;
    int ntiles = 0;
    int device = 0;
    double* scratch = nullptr;           // this device's copy of `scratch`
    // replay of a captured pair of steps (parity 0 -> 1 -> 0)
    int graph_steps = 0;                 // 0: plain launches
    hipGraphExec_t graph = nullptr;
    int graph_variant = -1;
};

namespace {

int32_t dev_err(hipError_t e) { return e == hipSuccess ? PFLBM_OK : PFLBM_ERR_DEVICE; }

int32_t build_tiles(pflbm_ctx* c, int v) {
    int tx, ty, nt;
    if (!step_variant_shape(v, c->prm[0].n_h, &tx, &ty, &nt)) return PFLBM_ERR_INVALID_ARG;
    std::vector<TileDev> tiles;
    for (int k = 0; k < (int)c->prm.size(); ++k) {
        const int nx = c->prm[k].nx, ny = c->prm[k].ny;
        for (int y0 = 0; y0 < ny; y0 += ty)
            for (int x0 = 0; x0 < nx; x0 += tx) tiles.push_back(TileDev{k, x0, y0, 0});
    }
    if (tiles.size() > c->L.max_tiles || tiles.empty()) return PFLBM_ERR_WORKSPACE;
    hipError_t e = hipMemcpyAsync(c->ws + c->L.tiles_off, tiles.data(), sizeof(TileDev) * tiles.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return PFLBM_ERR_DEVICE;
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return PFLBM_ERR_DEVICE;
    c->ntiles = (int)tiles.size();
    c->variant = v;
    return PFLBM_OK;
}

const CaseDev* dev_case(const pflbm_ctx* c, int k) {
    return reinterpret_cast<const CaseDev*>(c->ws + c->L.cases_off) + k;
}

unsigned int* dev_flags(const pflbm_ctx* c) { return reinterpret_cast<unsigned int*>(c->ws + c->L.flags_off); }

// Clears the non-finite flag of case k, or of every case for k < 0.
hipError_t clear_flags(pflbm_ctx* c, int k) {
    const int n = (int)c->prm.size();
    if (k < 0) {
        for (auto& v : c->nonfinite) v = 0;
        return launch_clear_flags(dev_flags(c), n, c->stream);
    }
    c->nonfinite[k] = 0;
    return launch_clear_flags(dev_flags(c) + k, 1, c->stream);
}

// True when a synchronising call has seen any case's non-finite flag set.
bool any_nonfinite(const pflbm_ctx* c) {
    for (int v : c->nonfinite)
        if (v) return true;
    return false;
}

bool all_init(const pflbm_ctx* c) {
    for (int v : c->initialised)
        if (!v) return false;
    return true;
}

}  // namespace

extern "C" {

size_t pflbm_workspace_bytes(const pflbm_params* cases, int32_t ncases) {
    Layout L;
    if (!make_layout(cases, ncases, &L)) return 0;
    return L.total;
}

int32_t pflbm_create(const pflbm_params* cases, int32_t ncases, void* d_workspace, size_t bytes, void* hip_stream,
                     pflbm_ctx** out) {
    if (!out) return PFLBM_ERR_INVALID_ARG;
    *out = nullptr;
    Layout L;
    if (!cases || ncases <= 0 || !make_layout(cases, ncases, &L)) return PFLBM_ERR_INVALID_ARG;
    if (cases[0].storage == 1 && cases[0].store_h) return PFLBM_ERR_UNSUPPORTED;
    // open ends are built for the compact state forms only
    for (int k = 0; k < ncases; ++k)
        if (cases[k].open_x && cases[k].store_h) return PFLBM_ERR_UNSUPPORTED;
    if (!d_workspace || bytes < L.total || ((uintptr_t)d_workspace % kAlign) != 0) return PFLBM_ERR_WORKSPACE;
    pflbm_ctx* c = new (std::nothrow) pflbm_ctx;
    if (!c) return PFLBM_ERR_DEVICE;
    c->prm.assign(cases, cases + ncases);
    c->L = L;
    c->ws = static_cast<char*>(d_workspace);
    c->ws_bytes = bytes;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->initialised.assign(ncases, 0);
    c->nonfinite.assign(ncases, 0);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return PFLBM_ERR_DEVICE; }
    if (scratch_address(c->device, &c->scratch) != hipSuccess) { delete c; return PFLBM_ERR_DEVICE; }
    c->cd.resize(ncases);
    for (int k = 0; k < ncases; ++k) {
        const pflbm_params& p = cases[k];
        const CaseLayout& cl = L.cl[k];
        CaseDev& d = c->cd[k];
        memset(&d, 0, sizeof(d));
        d.nx = p.nx; d.ny = p.ny; d.pitch = cl.pitch; d.n_h = p.n_h; d.plane = cl.plane;
        for (int b = 0; b < 2; ++b) {
            d.P[b] = reinterpret_cast<double*>(c->ws + cl.P[b]);
            d.S[b] = reinterpret_cast<float*>(c->ws + cl.S[b]);
            d.C[b] = reinterpret_cast<double*>(c->ws + cl.C[b]);
            d.T[b] = reinterpret_cast<float*>(c->ws + cl.T[b]);
            d.H[b] = p.store_h ? reinterpret_cast<float*>(c->ws + cl.H[b]) : nullptr;
            d.Q[b] = p.storage == 1 ? reinterpret_cast<_Float16*>(c->ws + cl.Q[b]) : nullptr;
        }
        d.qscale = kQScale;
        d.qinv = 1.0f / kQScale;
        for (int j = 0; j < 3; ++j) { d.rho[j] = (float)p.rho[j]; d.drho[j] = p.rho[j]; d.nu[j] = (float)p.nu[j]; d.inu[j] = (float)(1.0 / p.nu[j]); }
        d.plc = p.powerlaw_comp;
        d.nuloF = INFINITY;
        d.nuhiF = 0.0f;
        for (int j = 0; j < 3; ++j) {
            d.inuF[j] = j == d.plc ? 0.0f : d.inu[j];
            if (j != d.plc) { d.nuloF = std::min(d.nuloF, d.nu[j]); d.nuhiF = std::max(d.nuhiF, d.nu[j]); }
        }
        d.vm = p.variable_mobility ? 1 : 0;
        d.tau_iters = p.tau_iterations;
        d.hcd = p.hforce_cd;
        d.openx = p.open_x;
        d.u_in = (float)p.u_in;
        d.mflux = p.mobility_flux;
        d.K = (float)p.K; d.nexp = (float)p.n; d.numin = (float)p.nu_min; d.numax = (float)p.nu_max;
        d.sig12 = (float)p.sigma12; d.sig13 = (float)p.sigma13; d.sig23 = (float)p.sigma23; d.lam = (float)p.Lambda;
        double S[3], ST;
        capillary(p, S, &ST);
        for (int j = 0; j < 3; ++j) d.Sig[j] = (float)S[j];
        d.xi = (float)p.xi;
        d.mob[0] = (float)(p.D0 / S[0]);
        d.mob[1] = (float)(p.D0 / S[1]);
        d.omh = (float)(1.0 / (p.tau_h + 0.5));
        d.g = (float)p.g; d.fx = (float)p.fx;
        d.pref_g = (float)(p.rho[2] * p.g);
        d.pref_yc = (float)(0.5 * (p.ny - 1));
        d.dsig12 = p.sigma12; d.dsig13 = p.sigma13; d.dsig23 = p.sigma23; d.dlam = p.Lambda;
        for (int j = 0; j < 3; ++j) { d.dSig[j] = S[j]; d.dA[j] = 4.0 * ST / (p.xi * S[j]); }
        d.flag = reinterpret_cast<unsigned int*>(c->ws + L.flags_off) + k;
    }
    hipError_t e = hipMemcpyAsync(c->ws + L.cases_off, c->cd.data(), sizeof(CaseDev) * ncases, hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = clear_flags(c, -1);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { delete c; return PFLBM_ERR_DEVICE; }
    int32_t st = build_tiles(c, 0);
    if (st != PFLBM_OK) { delete c; return st; }
    *out = c;
    return PFLBM_OK;
}

int32_t pflbm_init_fields(pflbm_ctx* c, int32_t k, const double* C, const double* u, const double* p) {
    if (!c || k < 0 || k >= (int)c->prm.size() || !C) return PFLBM_ERR_INVALID_ARG;
    const pflbm_params& prm = c->prm[k];
    const size_t n = (size_t)prm.nx * prm.ny;
    for (size_t i = 0; i < n * prm.n_h; ++i) if (!is_finite(C[i])) return PFLBM_ERR_NONFINITE;
    if (u) for (size_t i = 0; i < 2 * n; ++i) if (!is_finite(u[i])) return PFLBM_ERR_NONFINITE;
    if (p) for (size_t i = 0; i < n; ++i) if (!is_finite(p[i])) return PFLBM_ERR_NONFINITE;
    double* st = reinterpret_cast<double*>(c->ws + c->L.staging_off);
    double* dC = st;
    double* du = st + n * prm.n_h;
    double* dp = du + 2 * n;
    hipError_t e = hipMemcpyAsync(dC, C, sizeof(double) * n * prm.n_h, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(du, u, sizeof(double) * 2 * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && p) e = hipMemcpyAsync(dp, p, sizeof(double) * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_init(dev_case(c, k), c->cd[k], c->par, dC, u ? du : nullptr, p ? dp : nullptr, c->stream);
    if (e == hipSuccess) e = clear_flags(c, k);
    // the staging area is reused by the next call: keep the host in step
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return PFLBM_ERR_DEVICE;
    c->initialised[k] = 1;
    return PFLBM_OK;
}

static hipError_t launch_one(pflbm_ctx* c, int par) {
    const CaseDev* cases = dev_case(c, 0);
    const TileDev* tiles = reinterpret_cast<const TileDev*>(c->ws + c->L.tiles_off);
    // the extended kernel instances when any case needs one of their features
    bool ext = false;
    for (const auto& p : c->prm) ext = ext || p.tau_iterations > 0 || p.hforce_cd || p.open_x || p.mobility_flux;
    const int form = (c->prm[0].storage == 1 ? 2 : (c->prm[0].store_h ? 1 : 0)) + (ext ? 3 : 0);
    return launch_step(c->variant, c->prm[0].n_h, form, cases, tiles, c->ntiles, par, c->stream);
}

static void drop_graph(pflbm_ctx* c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_variant = -1;
}

// Captures graph_steps launches (an even number, parities alternating from 0)
// on a private capture of the context's stream.
static int32_t build_graph(pflbm_ctx* c) {
    drop_graph(c);
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return PFLBM_ERR_DEVICE;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipStream_t saved = c->stream;
    c->stream = cs;
    for (int k = 0; e == hipSuccess && k < c->graph_steps; ++k) e = launch_one(c, k & 1);
    c->stream = saved;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) { c->graph = nullptr; return PFLBM_ERR_DEVICE; }
    c->graph_variant = c->variant;
    return PFLBM_OK;
}

int32_t pflbm_step(pflbm_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return PFLBM_ERR_INVALID_ARG;
    if (!all_init(c)) return PFLBM_ERR_STATE;
    int64_t s = 0;
    if (c->graph_steps > 0 && nsteps >= c->graph_steps) {
        if (!c->graph || c->graph_variant != c->variant) {
            int32_t st = build_graph(c);
            if (st != PFLBM_OK) return st;
        }
        // the graph starts from parity 0: bring the state there first
        if (c->par != 0) {
            if (launch_one(c, c->par) != hipSuccess) return PFLBM_ERR_DEVICE;
            c->par ^= 1;
            ++s;
        }
        for (; s + c->graph_steps <= nsteps; s += c->graph_steps)
            if (hipGraphLaunch(c->graph, c->stream) != hipSuccess) return PFLBM_ERR_DEVICE;
    }
    for (; s < nsteps; ++s) {
        if (launch_one(c, c->par) != hipSuccess) return PFLBM_ERR_DEVICE;
        c->par ^= 1;
    }
    return PFLBM_OK;
}

int32_t pflbm_set_graph(pflbm_ctx* c, int32_t steps_per_graph) {
    if (!c || steps_per_graph < 0 || (steps_per_graph & 1)) return PFLBM_ERR_INVALID_ARG;
    drop_graph(c);
    c->graph_steps = steps_per_graph;
    return PFLBM_OK;
}

int32_t pflbm_autotune(pflbm_ctx* c, int32_t steps, int32_t* best, float* ms_per_variant) {
    if (!c || steps <= 0) return PFLBM_ERR_INVALID_ARG;
    if (!all_init(c)) return PFLBM_ERR_STATE;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PFLBM_ERR_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return PFLBM_ERR_DEVICE; }
    int bestv = -1;
    float bestms = 0.f;
    int32_t st = PFLBM_OK;
    const int nv = step_variant_count();
    const int prev = c->variant;
    std::vector<float> best_ms(nv, -1.0f);
    // two passes over the variants, each variant's faster one counting: the
    // first variants timed would otherwise meet the GPU still ramping up
    for (int pass = 0; pass < 2 && st == PFLBM_OK; ++pass) {
        for (int v = 0; v < nv && st == PFLBM_OK; ++v) {
            int tx, ty, nt;
            if (!step_variant_shape(v, c->prm[0].n_h, &tx, &ty, &nt)) continue;
            st = build_tiles(c, v);
            if (st != PFLBM_OK) break;
            // every launch reads the current parity and writes the other buffer:
            // the state is left as it was
            hipError_t e = hipSuccess;
            for (int k = 0; k < 2 && e == hipSuccess; ++k) e = launch_one(c, c->par);
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            for (int k = 0; k < steps && e == hipSuccess; ++k) e = launch_one(c, c->par);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { st = PFLBM_ERR_DEVICE; break; }
            ms /= (float)steps;
            if (best_ms[v] < 0.0f || ms < best_ms[v]) best_ms[v] = ms;
        }
    }
    for (int v = 0; v < nv && st == PFLBM_OK; ++v) {
        if (ms_per_variant) ms_per_variant[v] = best_ms[v];
        if (best_ms[v] >= 0.0f && (bestv < 0 || best_ms[v] < bestms)) { bestv = v; bestms = best_ms[v]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PFLBM_OK) {
        (void)build_tiles(c, prev);   // best effort: leave the variant the call found
        return st;
    }
    if (best) *best = bestv;
    st = build_tiles(c, bestv);
    if (st == PFLBM_OK && any_nonfinite(c)) st = PFLBM_ERR_NONFINITE;
    return st;
}

int32_t pflbm_macroscopic(pflbm_ctx* c, int32_t k, float* rho, float* u, float* p, float* phi) {
    if (!c || k < 0 || k >= (int)c->prm.size()) return PFLBM_ERR_INVALID_ARG;
    if (!c->initialised[k]) return PFLBM_ERR_STATE;
    if (!rho && !u && !p && !phi) return PFLBM_OK;
    return dev_err(launch_macro(dev_case(c, k), c->cd[k], c->par, rho, u, p, phi, c->stream));
}

// The six sums of the bubble diagnostics of case k into out (shared by the
// workspace and the no-allocation entry points; `part` holds
// reduce_blocks() x 6 partials, `res` 6 results).
static int32_t centroid_sums(pflbm_ctx* c, int32_t k, int32_t comp, double* part, double* res, double out[6]) {
    hipError_t e = launch_reduce(dev_case(c, k), c->cd[k], c->par, comp, part, res, c->stream);
    double sums[6];
    unsigned int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(sums, res, sizeof(sums), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, dev_flags(c) + k, sizeof(flag), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return PFLBM_ERR_DEVICE;
    if (flag) c->nonfinite[k] = 1;
    if (c->nonfinite[k]) return PFLBM_ERR_NONFINITE;
    for (int j = 0; j < 6; ++j) if (!is_finite(sums[j])) return PFLBM_ERR_NONFINITE;
    // a component with no mass has no centroid or mean velocity
    if (sums[0] == 0.0) return PFLBM_ERR_NONFINITE;
    const double m = sums[0];
    out[0] = m;
    out[1] = sums[1];
    out[2] = sums[2] / m;
    out[3] = sums[3] / m;
    out[4] = sums[4] / m;
    out[5] = sums[5] / m;
    return PFLBM_OK;
}

int32_t pflbm_bubble_centroid_velocity(pflbm_ctx* c, int32_t k, int32_t comp, double out[6]) {
    if (!c || k < 0 || k >= (int)c->prm.size() || comp < 0 || comp > 2 || !out) return PFLBM_ERR_INVALID_ARG;
    if (comp == 1 && c->prm[k].n_h == 1) return PFLBM_ERR_INVALID_ARG;   // C_2 is not carried
    if (!c->initialised[k]) return PFLBM_ERR_STATE;
    double* res = reinterpret_cast<double*>(c->ws + c->L.result_off);
    double* part = reinterpret_cast<double*>(c->ws + c->L.partial_off);
    return centroid_sums(c, k, comp, part, res, out);
}

int32_t pflbm_bubble_centroid_velocity_noalloc(pflbm_ctx* c, int32_t k, int32_t comp, double out[6]) {
    if (!c || k < 0 || k >= (int)c->prm.size() || comp < 0 || comp > 2 || !out) return PFLBM_ERR_INVALID_ARG;
    if (comp == 1 && c->prm[k].n_h == 1) return PFLBM_ERR_INVALID_ARG;
    if (!c->initialised[k]) return PFLBM_ERR_STATE;
    // the partials of every reduction block and the 6 sums must fit the
    // static scratch (the reduction caps its grid at kReduceMax blocks, so
    // every domain size fits; the check guards the layout)
    const int nb = reduce_blocks(c->cd[k]);
    if (nb <= 0 || (size_t)nb * 6 + 8 > kScratchDoubles) return PFLBM_ERR_WORKSPACE;
    double* part = c->scratch;
    double* res = c->scratch + 6 * (size_t)kReduceMax;
    return centroid_sums(c, k, comp, part, res, out);
}

int32_t pflbm_check_state(pflbm_ctx* c) {
    if (!c) return PFLBM_ERR_INVALID_ARG;
    if (!all_init(c)) return PFLBM_ERR_STATE;
    const int n = (int)c->prm.size();
    hipError_t e = hipSuccess;
    for (int k = 0; k < n && e == hipSuccess; ++k) e = launch_check(dev_case(c, k), c->cd[k], c->par, c->stream);
    std::vector<unsigned int> flags(n, 0u);
    if (e == hipSuccess)
        e = hipMemcpyAsync(flags.data(), dev_flags(c), sizeof(unsigned int) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return PFLBM_ERR_DEVICE;
    for (int k = 0; k < n; ++k)
        if (flags[k]) c->nonfinite[k] = 1;
    return any_nonfinite(c) ? PFLBM_ERR_NONFINITE : PFLBM_OK;
}

int32_t pflbm_case_nonfinite(const pflbm_ctx* c, int32_t k) {
    if (!c || k < 0 || k >= (int)c->prm.size()) return PFLBM_ERR_INVALID_ARG;
    return c->nonfinite[k] ? 1 : 0;
}

size_t pflbm_state_bytes(const pflbm_ctx* c) {
    if (!c) return 0;
    size_t b = 0;
    for (size_t k = 0; k < c->prm.size(); ++k) b += c->L.cl[k].P[1] - c->L.cl[k].P[0];
    return b;
}

static int32_t copy_state(pflbm_ctx* c, char* dst, const char* src, bool to_ws) {
    size_t o = 0;
    for (size_t k = 0; k < c->prm.size(); ++k) {
        const CaseLayout& cl = c->L.cl[k];
        const size_t len = cl.P[1] - cl.P[0];
        char* w = c->ws + cl.P[c->par];
        hipError_t e = to_ws ? hipMemcpyAsync(w, src + o, len, hipMemcpyDeviceToDevice, c->stream)
                             : hipMemcpyAsync(dst + o, w, len, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return PFLBM_ERR_DEVICE;
        o += len;
    }
    return PFLBM_OK;
}

int32_t pflbm_get_state(pflbm_ctx* c, void* d_dst, size_t bytes) {
    if (!c || !d_dst) return PFLBM_ERR_INVALID_ARG;
    if (bytes < pflbm_state_bytes(c)) return PFLBM_ERR_WORKSPACE;
    return copy_state(c, static_cast<char*>(d_dst), nullptr, false);
}

int32_t pflbm_set_state(pflbm_ctx* c, const void* d_src, size_t bytes) {
    if (!c || !d_src) return PFLBM_ERR_INVALID_ARG;
    if (bytes < pflbm_state_bytes(c)) return PFLBM_ERR_WORKSPACE;
    int32_t st = copy_state(c, nullptr, static_cast<const char*>(d_src), true);
    if (st == PFLBM_OK && clear_flags(c, -1) != hipSuccess) st = PFLBM_ERR_DEVICE;
    if (st == PFLBM_OK) for (auto& v : c->initialised) v = 1;
    return st;
}

int32_t pflbm_export_populations(pflbm_ctx* c, int32_t k, float* d_out) {
    if (!c || k < 0 || k >= (int)c->prm.size() || !d_out) return PFLBM_ERR_INVALID_ARG;
    if (!c->initialised[k]) return PFLBM_ERR_STATE;
    return dev_err(launch_export(dev_case(c, k), c->cd[k], c->par, d_out, c->stream));
}

int32_t pflbm_num_variants(const pflbm_ctx* c) { return c ? step_variant_count() : 0; }

const char* pflbm_variant_name(const pflbm_ctx* c, int32_t v) {
    static thread_local char buf[64];
    int tx, ty, nt;
    if (!c || !step_variant_shape(v, c->prm[0].n_h, &tx, &ty, &nt)) return nullptr;
    snprintf(buf, sizeof(buf), "tile%dx%d_t%d", tx, ty, nt);
    return buf;
}

int32_t pflbm_set_variant(pflbm_ctx* c, int32_t v) {
    if (!c) return PFLBM_ERR_INVALID_ARG;
    if (v == -1) v = 0;
    return build_tiles(c, v);
}

void* pflbm_stream(const pflbm_ctx* c) { return c ? (void*)c->stream : nullptr; }

double pflbm_bytes_per_update(const pflbm_ctx* c) {
    if (!c) return 0.0;
    const pflbm_params& p = c->prm[0];
    // gbar: s (float64) + 8 deviations (float32), or s (float64) + j_x, j_y
    // (float32) + 6 pair moments (float16); C_i (float64); tau (float32);
    // hbar deviations (float32) when stored
    double b = 8 + (p.storage == 1 ? 2 * 4 + 6 * 2 : 8 * 4) + 8.0 * p.n_h + 4;
    if (p.store_h) b += 9 * 4.0 * p.n_h;
    return 2.0 * b;                        // read once and written once
}

int32_t pflbm_destroy(pflbm_ctx* c) {
    if (!c) return PFLBM_ERR_INVALID_ARG;
    drop_graph(c);
    const hipError_t e = hipStreamSynchronize(c->stream);
    delete c;
    if (e != hipSuccess) return PFLBM_ERR_DEVICE;
    return PFLBM_OK;
}

const char* pflbm_status_string(int32_t s) {
    switch (s) {
        case PFLBM_OK: return "ok";
        case PFLBM_ERR_INVALID_ARG: return "invalid argument";
        case PFLBM_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
        case PFLBM_ERR_DEVICE: return "HIP device error";
        case PFLBM_ERR_NONFINITE: return "non-finite value";
        case PFLBM_ERR_STATE: return "call out of order";
        case PFLBM_ERR_UNSUPPORTED: return "unsupported by the library";
        default: return "unknown status";
    }
}

}  // extern "C"
