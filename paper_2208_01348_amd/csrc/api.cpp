// C ABI of the gfx950 DDA library (declared in include/dda.h) and the host
// orchestration of its kernels.
#include "dda.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <cmath>
#include <limits>
#include <complex>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "krylov.h"

using dda::Error;
using dda::z128;
using dda::z64;
using cplx = std::complex<double>;

namespace {

thread_local std::string g_last_error;

constexpr double kHbarC = 197.3269804;        // eV nm
constexpr double kAlphaFs = 7.2973525693e-3;  // fine-structure constant
constexpr double kMeC2 = 510.99895;           // keV
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxSide = 256;
constexpr int kMaxRestarts = 20;
constexpr double kInnerTol = 1e-4;   // relative tolerance of the FP32 inner solves
constexpr int kMaxOuter = 60;
// QMR in FP32: a cycle stops when its residual bound has fallen this far below
// the residual it started from (the FP32 recursion resolves no more); the FP64
// check then restarts it from the new residual.
constexpr double kQmrInner = 1e-4;
// COCG folds an iteration's finalizer into the next direction update up to
// this many slots per launch (measured: a single solve 3.7 % faster, a
// 52-slot spectrum batch 2.5 % slower with the fold)
constexpr int kCocgFoldMaxSlots = 8;
// BiCGStab folds its p and s updates into the x kernels of the two matvecs up
// to this many slots per launch
constexpr int kBicgFoldMaxSlots = 8;

// ------------------------------------------------------------------ memory
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t n) {
        if (n <= bytes && p) return;
        release();
        if (n == 0) n = 256;
        DDA_HIP_CHECK(hipMalloc(&p, n));
        bytes = n;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
    void ensure(size_t n) {
        if (n <= bytes && p) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        DDA_HIP_CHECK(hipHostMalloc(&p, std::max<size_t>(n, 256), hipHostMallocDefault));
        bytes = std::max<size_t>(n, 256);
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// D(k) for one host wavenumber: FP64 always, FP32 copy on demand.
struct DEntry {
    DevBuf d128, d64;
    bool has64 = false;
    uint64_t last_use = 0;
    int refs = 0;  // engine slots solving at this wavenumber
};

struct Timer {
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double total_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t units[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    ~Timer() {
        for (auto& e : pool) (void)hipEventDestroy(e);
        for (auto& p : pending) {
            (void)hipEventDestroy(p.second.first);
            (void)hipEventDestroy(p.second.second);
        }
    }
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        DDA_HIP_CHECK(hipEventCreate(&e));
        return e;
    }
};

constexpr int kNumKernels = 8;
const char* const kKernelNames[kNumKernels] = {"unpack_xfft", "yfft",   "zconv",
                                               "iyfft",       "ixfft_pack", "yzconv",
                                               "xyfft",       "ixyfft_pack"};

int choose_fft_len(int n) {
    static const int sizes[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
    for (int s : sizes)
        if (s >= 2 * n - 1) return s;
    return -1;
}

cplx gamma_h_of(double beta, cplx mh) {
    // gamma_h = i / sqrt(beta_h^2 - 1), principal root; beta_h^2 - 1 lies in
    // the closed upper half plane for a passive host (eq. 24), and a zero
    // imaginary part is taken as +0.
    cplx bh = beta * mh;
    cplx w = bh * bh - 1.0;
    if (std::abs(w) < 1e-12)
        throw Error(DDA_ESINGULAR, "beta_h = 1: the electron field is singular (eq. 24)");
    if (w.imag() == 0.0) w = cplx(w.real(), 0.0);
    cplx sq = (w.imag() == 0.0 && w.real() < 0.0) ? cplx(0.0, std::sqrt(-w.real())) : std::sqrt(w);
    return cplx(0.0, 1.0) / sq;
}

// Spins until an event has completed (an event never recorded counts as
// complete).
void wait_event(hipEvent_t e) {
    hipError_t r;
    while ((r = hipEventQuery(e)) == hipErrorNotReady) {
    }
    DDA_HIP_CHECK(r);
}

// Pinned staging with kRing regions, so that an upload or a state snapshot
// can be in flight while the host fills the next region.
constexpr int kRing = 4;

// Active lists uploaded in stream order; a region is refilled only after its
// previous copy has run.
struct ActRing {
    DevBuf dev;  // the list the kernels read
    PinnedBuf host;
    hipEvent_t ev[kRing] = {};
    int seq = 0, cap = 0;
    ActRing() = default;
    ActRing(const ActRing&) = delete;
    ~ActRing() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void ensure(int n) {
        dev.ensure(size_t(n) * sizeof(int));
        if (n > cap) {
            for (auto e : ev)
                if (e) wait_event(e);  // copies in flight read the old buffer
            cap = n;
        }
        host.ensure(size_t(kRing) * cap * sizeof(int));
    }
    void upload(hipStream_t s, const std::vector<int>& act) {
        if (act.empty()) return;
        if (int(act.size()) > cap) throw Error(DDA_EDEVICE, "active list larger than its buffer");
        const int r = seq++ % kRing;
        if (!ev[r]) DDA_HIP_CHECK(hipEventCreateWithFlags(&ev[r], hipEventDisableTiming));
        wait_event(ev[r]);
        int* h = host.as<int>() + size_t(r) * cap;
        std::memcpy(h, act.data(), act.size() * sizeof(int));
        DDA_HIP_CHECK(hipMemcpyAsync(dev.p, h, act.size() * sizeof(int), hipMemcpyHostToDevice, s));
        DDA_HIP_CHECK(hipEventRecord(ev[r], s));
    }
    const int* ptr() const { return dev.as<int>(); }
};

// Slot states copied to pinned memory after every interval k (region
// k mod kRing); read back kLag intervals later without stalling the stream.
struct StateRing {
    PinnedBuf host;
    hipEvent_t ev[kRing] = {};
    int cap = 0;
    StateRing() = default;
    StateRing(const StateRing&) = delete;
    ~StateRing() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void ensure(int n) {
        if (n > cap) {
            for (auto e : ev)
                if (e) wait_event(e);
            cap = n;
        }
        host.ensure(size_t(kRing) * cap * sizeof(dda::BicgSlot));
        for (auto& e : ev)
            if (!e) DDA_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    void snapshot(hipStream_t s, const dda::BicgSlot* st, int n, int64_t k) {
        const int r = int(k % kRing);
        DDA_HIP_CHECK(hipMemcpyAsync(host.as<dda::BicgSlot>() + size_t(r) * cap, st,
                                     size_t(n) * sizeof(dda::BicgSlot), hipMemcpyDeviceToHost, s));
        DDA_HIP_CHECK(hipEventRecord(ev[r], s));
    }
    const dda::BicgSlot* wait(int64_t k) {
        const int r = int(k % kRing);
        wait_event(ev[r]);
        return host.as<dda::BicgSlot>() + size_t(r) * cap;
    }
};

// Tile choices of the matvec chain for one precision, picked by timing the
// candidates (autotune); 0 means the compiled-in default.
struct TuneVal {
    bool done = false;
    int zconv_tx = 0, mid_tx = 0, yz_threads = 0;
    double t_default_ms = 0.0, t_best_ms = 0.0;  // the tuned kernel, default vs chosen
};

// Choices shared by every context of the process with the same lattice and
// FFT grid, so that they all run the same kernels.
std::mutex g_tune_mu;
std::map<std::array<int, 7>, TuneVal> g_tune;

// A captured interval, replayed while its key (the active-list length) holds.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int key = -1;
    GraphCache() = default;
    GraphCache(const GraphCache&) = delete;
    ~GraphCache() { drop(); }
    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key = -1;
    }
};

}  // namespace

struct dda_ctx {
    dda::Geo g{};
    double d = 1.0;
    cplx mh;
    dda_options opt{};
    hipStream_t stream = nullptr;
    std::vector<int> occ_lin;  // host copy
    std::vector<char> occ_col;  // [ny][nx]: the (x, y) column holds a dipole
    int device = 0;             // the device current at dda_setup
    DevBuf map, occ;
    DevBuf tw128[3], tw64[3];
    std::map<std::pair<double, double>, std::unique_ptr<DEntry>> dcache;
    // evicted entries whose buffers the next misses reuse: freeing device
    // memory waits for the whole device, which stalls every other stream's
    // host thread in a multi-lattice server; every reader of a D is on this
    // context's stream, so a reused buffer is rewritten only after them
    std::vector<std::unique_ptr<DEntry>> dspare;
    uint64_t use_clock = 0;
    uint64_t pin_clock = 0;   // entries used at or after this tick are in use
    size_t dcache_limit = size_t(64) << 30;
    // work space
    DevBuf G, vec128, vec64, st, partial, slot_sys, dptr, ainv128, ainv64, misc;
    DevBuf dfull;  // scratch of the full-grid transform during a D build
    DevBuf igt_buf;      // integrated interaction: near offsets and the cubature rule
    dda::IgtTable igt{};
    DevBuf eps_dev, matsys;  // permittivities and wavenumbers of a chunk
    DevBuf ff_coord, ff_buf;  // far-field: packed dipole coordinates, work space
    PinnedBuf host_st, host_misc;
    ActRing act;
    StateRing ring;
    // Captured COCG interval (not used while kernels are timed: events
    // recorded by graph nodes carry no timestamps)
    GraphCache graph;
    TuneVal tune[2];  // [0] FP32, [1] FP64 matvec chain
    std::unique_ptr<struct Engine> engine;  // continuous batching, when open
    int max_blocks = 1024;
    bool timing = false;
    unsigned timing_mask = 0xff;  // which matvec kernels are timed
    Timer timer;
    hipEvent_t sync_ev = nullptr;  // for low-latency host waits

    int64_t nv() const { return 3 * g.n_occ; }
};

namespace {

template <typename T>
const dda::cx<T>* tw_of(const dda_ctx* c, int axis);
template <>
const z128* tw_of<double>(const dda_ctx* c, int axis) { return c->tw128[axis].as<z128>(); }
template <>
const z64* tw_of<float>(const dda_ctx* c, int axis) { return c->tw64[axis].as<z64>(); }

void check_finite(double v, const char* what) {
    if (!std::isfinite(v)) throw Error(DDA_EINVAL, std::string(what) + " is not finite");
}

// Waits until the context's stream has drained, spinning on an event: the
// solver loop waits for a few scalars every few iterations, and a sleeping
// wait costs about a millisecond of wake-up latency each time.
void wait_stream(dda_ctx* c) {
    if (!c->sync_ev)
        DDA_HIP_CHECK(hipEventCreateWithFlags(&c->sync_ev, hipEventDisableTiming));
    DDA_HIP_CHECK(hipEventRecord(c->sync_ev, c->stream));
    hipError_t e;
    while ((e = hipEventQuery(c->sync_ev)) == hipErrorNotReady) {
    }
    DDA_HIP_CHECK(e);
}

// Copies a pageable host array to the device in the order of the context's
// stream and waits for it (the host array may go out of scope afterwards).
void upload(dda_ctx* c, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return;
    DDA_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    wait_stream(c);
}

struct Tic {
    dda_ctx* c;
    int k;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    Tic(dda_ctx* c_, int k_, int n_rhs) : c(c_), k(k_), on(c_->timing && ((c_->timing_mask >> k_) & 1u)) {
        if (on) {
            c->timer.units[k] += n_rhs;
            a = c->timer.get();
            b = c->timer.get();
            DDA_HIP_CHECK(hipEventRecord(a, c->stream));
        }
    }
    ~Tic() {
        if (on) {
            (void)hipEventRecord(b, c->stream);
            c->timer.pending.push_back({k, {a, b}});
        }
    }
};

void flush_timer(dda_ctx* c) {
    if (c->timer.pending.empty()) return;
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
    for (auto& p : c->timer.pending) {
        float ms = 0.f;
        DDA_HIP_CHECK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        c->timer.total_ms[p.first] += ms;
        c->timer.count[p.first] += 1;
        c->timer.pool.push_back(p.second.first);
        c->timer.pool.push_back(p.second.second);
    }
    c->timer.pending.clear();
}

// Graph capture is used when enabled and no per-kernel timing is requested.
bool use_graphs(const dda_ctx* c) {
    return c->opt.use_graphs != 0 && c->stream != nullptr && !c->timing;
}

// Launches body() on the context's stream through the captured graph in gc:
// replayed while `key` is unchanged, captured again otherwise (the executable
// is updated in place when the topology allows it, else instantiated anew).
template <typename F>
void launch_captured(dda_ctx* c, GraphCache& gc, int key, F&& body) {
    hipStream_t s = c->stream;
    if (!gc.exec || gc.key != key) {
        hipGraph_t gr = nullptr;
        DDA_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(s, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
            throw;
        }
        DDA_HIP_CHECK(hipStreamEndCapture(s, &gr));
        bool updated = false;
        if (gc.exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res;
            updated = hipGraphExecUpdate(gc.exec, gr, &bad, &res) == hipSuccess &&
                      res == hipGraphExecUpdateSuccess;
            if (!updated) {
                (void)hipGetLastError();
                gc.drop();
            }
        }
        hipError_t e = hipSuccess;
        if (!updated) e = hipGraphInstantiate(&gc.exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        DDA_HIP_CHECK(e);
        gc.key = key;
    }
    DDA_HIP_CHECK(hipGraphLaunch(gc.exec, s));
}

dda::RedScratch red_of(dda_ctx* c) {
    return dda::RedScratch{c->partial.as<double>(), c->max_blocks};
}

// Buffers a solver driver works in: slot states, reduction rows and the grid
// work buffer of the matvec (indexed by active-list position).
struct Work {
    dda::BicgSlot* st;
    dda::RedScratch red;
    void* G;
    const int* map = nullptr;  // per-slot index maps (slot s at map + s * map_stride), or
    int64_t map_stride = 0;    // nullptr: the context's own map for every slot
};
Work ctx_work(dda_ctx* c) { return Work{c->st.as<dda::BicgSlot>(), red_of(c), c->G.p}; }

// Picks the tile widths of the chain for precision T by timing every
// candidate on up to 8 of the listed right-hand sides (HIP events, best of
// three after a warm-up): the threads per block of the fused yz kernel, or
// the columns per block of the z-convolution and y passes of the five-pass
// chain (the z pass alone in the fused xy chain).  The candidates differ only in how lines are grouped into blocks, so
// the choice never changes a result.  Runs once per process and geometry
// (never inside a stream capture: there the defaults stand until tuning has
// run outside one); it writes only the grid work buffer, which every matvec
// rewrites before reading.
template <typename T>
void autotune(dda_ctx* c, const Work& w, const int* act, int n_act,
              const dda::cx<T>* const* dptr, const int* slot_sys) {
    constexpr int csize = int(sizeof(dda::cx<T>));
    TuneVal& tv = c->tune[csize == 16 ? 1 : 0];
    if (tv.done || n_act == 0 || c->g.n_occ == 0) return;
    const dda::Geo& g = c->g;
    const std::array<int, 7> key{g.nx, g.ny, g.nz, g.mx, g.my, g.mz, csize};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            tv = it->second;
            return;
        }
    }
    hipStream_t s = c->stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DDA_HIP_CHECK(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return;
    const int n = std::min(n_act, 8);
    auto* G = static_cast<dda::cx<T>*>(w.G);
    const dda::SlotFilter all{nullptr, dda::FILTER_ALL};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DDA_HIP_CHECK(hipEventCreate(&e0));
    DDA_HIP_CHECK(hipEventCreate(&e1));
    auto time_of = [&](auto&& launch) {
        launch();
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            DDA_HIP_CHECK(hipEventRecord(e0, s));
            launch();
            DDA_HIP_CHECK(hipEventRecord(e1, s));
            DDA_HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            DDA_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return double(best);
    };
    // the fastest candidate; returns {choice, default width's time, best time}
    // (choice 0 keeps the default: no candidate beat it)
    auto pick = [&](const std::vector<int>& cands, auto&& launch_with) {
        if (cands.empty()) return std::array<double, 3>{0.0, 0.0, 0.0};  // nothing to choose
        const double t_def = time_of([&] { launch_with(0); });
        int best_v = 0;
        double best_t = t_def;
        for (int v : cands) {
            const double t = time_of([&] { launch_with(v); });
            if (t < best_t) {
                best_t = t;
                best_v = v;
            }
        }
        return std::array<double, 3>{double(best_v), t_def, best_t};
    };
    TuneVal r;
    r.done = true;
    try {
        if (dda::yz_fused_ok(g, csize)) {
            const auto res = pick(dda::yz_thread_candidates(g.my), [&](int nt) {
                dda::launch_yzconv<T>(G, dptr, tw_of<T>(c, 1), tw_of<T>(c, 2), g, act, slot_sys, n,
                                      all, nt, s);
            });
            r.yz_threads = int(res[0]);
            r.t_default_ms = res[1];
            r.t_best_ms = res[2];
        } else {
            const auto rz = pick(dda::zconv_tx_candidates<T>(g.mz), [&](int tx) {
                dda::launch_zconv<T>(G, dptr, tw_of<T>(c, 2), g, act, slot_sys, n, all, tx, s);
            });
            r.zconv_tx = int(rz[0]);
            if (!dda::xy_fused_ok(g, csize)) {  // the fused xy chain has no y pass
                const int64_t plane = int64_t(g.my) * g.mx;
                const auto rm = pick(dda::mid_tx_candidates<T>(g.my), [&](int tx) {
                    dda::launch_fft_mid<T>(G, tw_of<T>(c, 1), g.my, false, int64_t(n) * 3 * g.nz,
                                           g.mx, g.ny, g.my, plane, tx, s);
                });
                r.mid_tx = int(rm[0]);
            }
            r.t_default_ms = rz[1];
            r.t_best_ms = rz[2];
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.emplace(key, r);
    }
    tv = r;
}

// One FFT matvec for the slots listed in act (device) / n_act:
// mode PACK_AX (y = A x), PACK_GX (y = G_off x) or PACK_AX_COCG (y = A x with
// the COCG scalars fused; then fuse_r gives the direction update
// x <- fuse_r + beta x done in place by the first kernel).
// Partial rows per slot of the fused pack modes, and of the x kernel (the
// rows of a folded BiCGStab s update), for the chain a precision runs: the
// three-pass chain, the fused xy chain (FP32 on 96- or 128-point x-y grids)
// or the five-pass chain.
int pack_blocks(const dda_ctx* c, int csize) {
    if (dda::yz_fused_ok(c->g, csize)) return dda::yz_pack_blocks_per_slot(c->g, csize);
    if (dda::xy_fused_ok(c->g, csize)) return dda::xy_pack_blocks_per_slot(c->g);
    return dda::pack_blocks_per_slot(c->g, csize);
}
int x_blocks(const dda_ctx* c, int csize) {
    if (dda::xy_fused_ok(c->g, csize)) return dda::xy_pack_blocks_per_slot(c->g);
    return dda::xfft_blocks_per_slot(c->g, csize);
}

template <typename T>
void matvec(dda_ctx* c, const Work& w, dda::cx<T>* x, dda::cx<T>* y, const int* act, int n_act,
            const dda::cx<T>* const* dptr, const int* slot_sys, const dda::cx<T>* ainv, int mode,
            const dda::cx<T>* fuse_r = nullptr,
            dda::SlotFilter f = dda::SlotFilter{nullptr, dda::FILTER_ALL},
            const dda::cx<T>* dotw = nullptr, dda::CocgFold fold = dda::CocgFold{},
            dda::BicgFold bfold = dda::BicgFold{}) {
    if (n_act == 0 || c->g.n_occ == 0) return;
    if (((fuse_r && bfold.kind == dda::BICG_FOLD_NONE) || f.mode != dda::FILTER_ALL) && !f.st)
        throw Error(DDA_EDEVICE, "slot filter without slot states");
    dda::Geo g = c->g;
    const int* map = c->map.as<int>();
    if (w.map) {
        map = w.map;
        g.map_stride = w.map_stride;
    }
    auto* G = static_cast<dda::cx<T>*>(w.G);
    hipStream_t s = c->stream;
    constexpr int csize = int(sizeof(dda::cx<T>));
    autotune<T>(c, w, act, n_act, dptr, slot_sys);
    const TuneVal& tn = c->tune[csize == 16 ? 1 : 0];
    if (dda::yz_fused_ok(g, csize)) {
        {
            Tic t(c, 0, n_act);
            dda::launch_xfft_t<T>(x, map, G, tw_of<T>(c, 0), g, act, n_act, fuse_r,
                                  f, s, fold, bfold);
        }
        {
            Tic t(c, 5, n_act);
            dda::launch_yzconv<T>(G, dptr, tw_of<T>(c, 1), tw_of<T>(c, 2), g, act, slot_sys, n_act,
                                  f, tn.yz_threads, s);
        }
        {
            Tic t(c, 4, n_act);
            dda::launch_ixfft_t<T>(G, x, ainv, y, map, tw_of<T>(c, 0), g, act,
                                   slot_sys, n_act, mode, f, w.red, s, dotw);
        }
    } else if (dda::xy_fused_ok(g, csize)) {
        {
            Tic t(c, 6, n_act);
            dda::launch_xyfft<T>(x, map, G, tw_of<T>(c, 0), g, act, n_act, fuse_r, f, s, fold,
                                 bfold);
        }
        {
            Tic t(c, 2, n_act);
            dda::launch_zconv<T>(G, dptr, tw_of<T>(c, 2), g, act, slot_sys, n_act, f, tn.zconv_tx,
                                 s);
        }
        {
            Tic t(c, 7, n_act);
            dda::launch_ixyfft_pack<T>(G, x, ainv, y, map, tw_of<T>(c, 0), g, act, slot_sys, n_act,
                                       mode, f, w.red, s, dotw);
        }
    } else {
        const int64_t plane = int64_t(g.my) * g.mx;
        {
            Tic t(c, 0, n_act);
            dda::launch_unpack_xfft<T>(x, map, G, tw_of<T>(c, 0), g, act, n_act,
                                       fuse_r, f, s, fold, bfold);
        }
        {
            Tic t(c, 1, n_act);
            dda::launch_fft_mid<T>(G, tw_of<T>(c, 1), g.my, false, int64_t(n_act) * 3 * g.nz,
                                   g.mx, g.ny, g.my, plane, tn.mid_tx, s);
        }
        {
            Tic t(c, 2, n_act);
            dda::launch_zconv<T>(G, dptr, tw_of<T>(c, 2), g, act, slot_sys, n_act, f, tn.zconv_tx,
                                 s);
        }
        {
            Tic t(c, 3, n_act);
            dda::launch_fft_mid<T>(G, tw_of<T>(c, 1), g.my, true, int64_t(n_act) * 3 * g.nz,
                                   g.mx, g.my, g.ny, plane, tn.mid_tx, s);
        }
        {
            Tic t(c, 4, n_act);
            dda::launch_ixfft_pack<T>(G, x, ainv, y, map, tw_of<T>(c, 0), g, act,
                                      slot_sys, n_act, mode, f, w.red, s, dotw);
        }
    }
}

template <typename T>
void matvec(dda_ctx* c, dda::cx<T>* x, dda::cx<T>* y, const int* act, int n_act,
            const dda::cx<T>* const* dptr, const int* slot_sys, const dda::cx<T>* ainv, int mode,
            const dda::cx<T>* fuse_r = nullptr,
            dda::SlotFilter f = dda::SlotFilter{nullptr, dda::FILTER_ALL},
            const dda::cx<T>* dotw = nullptr, dda::CocgFold fold = dda::CocgFold{},
            dda::BicgFold bfold = dda::BicgFold{}) {
    matvec<T>(c, ctx_work(c), x, y, act, n_act, dptr, slot_sys, ainv, mode, fuse_r, f, dotw, fold,
              bfold);
}

// ------------------------------------------------------------ D cache
// Stored D layout of a precision's matvec path: kx slabs for the three-pass
// chain, the [0, M/2]^3 corner otherwise.
bool uses_yz(const dda_ctx* c, int csize) { return dda::yz_fused_ok(c->g, csize); }
size_t d_elems(const dda_ctx* c, int csize) {
    return size_t(uses_yz(c, csize) ? dda::dyz_elems(c->g) : dda::dred_elems(c->g));
}

void build_full_D(dda_ctx* c, cplx k) {
    c->dfull.ensure(size_t(dda::dgrid_elems(c->g)) * sizeof(z128));
    const dda::IgtTable* igt = nullptr;
    if (c->opt.interaction == DDA_INT_IGT) {
        if (!c->igt.rule) {
            std::vector<int> off;
            std::vector<double> rule;
            dda::igt_host_tables(c->g, off, rule);
            const size_t ob = off.size() * sizeof(int), rb = rule.size() * sizeof(double);
            c->igt_buf.ensure(ob + rb + 256);
            char* base = c->igt_buf.as<char>();
            upload(c, base, rule.data(), rb);
            if (ob) upload(c, base + rb, off.data(), ob);
            c->igt.rule = reinterpret_cast<const double*>(base);
            c->igt.off = reinterpret_cast<const int*>(base + rb);
            c->igt.n = int(off.size() / 4);
        }
        igt = &c->igt;
    }
    dda::launch_build_D(c->dfull.as<z128>(), c->g, c->d, k.real(), k.imag(),
                        c->tw128[0].as<z128>(), c->tw128[1].as<z128>(), c->tw128[2].as<z128>(),
                        c->stream, igt);
}

template <typename T>
void extract_D(dda_ctx* c, dda::cx<T>* out) {
    if (uses_yz(c, int(sizeof(dda::cx<T>))))
        dda::launch_extract_yz<T>(c->dfull.as<z128>(), out, c->g, c->stream);
    else
        dda::launch_extract_corner<T>(c->dfull.as<z128>(), out, c->g, c->stream);
}

// D(k) from the cache, built on a miss (and its FP32 copy if need64).
DEntry* get_D_k(dda_ctx* c, cplx k, bool need64) {
    auto key = std::make_pair(k.real(), k.imag());
    auto it = c->dcache.find(key);
    DEntry* e;
    bool full_ready = false;
    if (it == c->dcache.end()) {
        const size_t b128 = d_elems(c, 16) * sizeof(z128);
        // evict least recently used entries beyond the limit
        size_t used = 0;
        for (auto& kv : c->dcache) used += kv.second->d128.bytes + kv.second->d64.bytes;
        while (used + b128 * 2 > c->dcache_limit) {
            auto victim = c->dcache.end();
            for (auto i2 = c->dcache.begin(); i2 != c->dcache.end(); ++i2)
                if (i2->second->last_use < c->pin_clock && i2->second->refs == 0 &&
                    (victim == c->dcache.end() || i2->second->last_use < victim->second->last_use))
                    victim = i2;
            if (victim == c->dcache.end()) break;  // everything cached is in use
            used -= victim->second->d128.bytes + victim->second->d64.bytes;
            if (c->dspare.size() < 2) c->dspare.push_back(std::move(victim->second));
            c->dcache.erase(victim);
        }
        std::unique_ptr<DEntry> ne;
        if (!c->dspare.empty()) {
            ne = std::move(c->dspare.back());
            c->dspare.pop_back();
            ne->has64 = false;
            ne->refs = 0;
        } else {
            ne = std::make_unique<DEntry>();
        }
        ne->d128.ensure(b128);
        build_full_D(c, k);
        full_ready = true;
        extract_D<double>(c, ne->d128.as<z128>());
        e = ne.get();
        c->dcache[key] = std::move(ne);
    } else {
        e = it->second.get();
    }
    if (need64 && !e->has64) {
        e->d64.ensure(d_elems(c, 8) * sizeof(z64));
        if (!full_ready) build_full_D(c, k);
        extract_D<float>(c, e->d64.as<z64>());
        e->has64 = true;
    }
    e->last_use = ++c->use_clock;
    return e;
}

DEntry* get_D(dda_ctx* c, double energy, bool need64) {
    return get_D_k(c, c->mh * (energy / kHbarC), need64);
}

// ------------------------------------------------------------ material terms
// True when p points to device memory (a pageable host pointer is unknown to
// the runtime and counts as host memory).
bool is_device_ptr(const void* p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// Copies the permittivities of systems [e0, e0 + ns) to the device and
// evaluates there, per dipole, 1/alpha (FP64 if need128, FP32 if need64) and,
// if w_dev is given, the absorption weight [ns][n_occ].  A non-finite
// permittivity or a vanishing or infinite polarizability is an EINVAL error
// before any solve runs.
void compute_material(dda_ctx* c, const double* energy, const double* eps, int e0, int ns,
                      bool need128, bool need64, double* w_dev) {
    const int64_t n = c->g.n_occ;
    const size_t cnt = size_t(ns) * size_t(n);
    if (cnt == 0) return;
    c->eps_dev.ensure(cnt * sizeof(z128));  // staging for a host array
    std::vector<dda::MatSys> hs(ns);
    for (int i = 0; i < ns; ++i) {
        const cplx k = c->mh * (energy[e0 + i] / kHbarC);
        hs[i] = dda::MatSys{k.real(), k.imag(), c->mh.real(), c->mh.imag()};
    }
    const size_t sb = hs.size() * sizeof(dda::MatSys);
    const size_t sb_al = (sb + 255) / 256 * 256;
    c->matsys.ensure(sb_al + size_t(ns) * sizeof(int));
    int* err = reinterpret_cast<int*>(c->matsys.as<char>() + sb_al);
    const z128* eps_dev = reinterpret_cast<const z128*>(eps) + int64_t(e0) * n;
    if (!is_device_ptr(eps)) {  // host array: upload the chunk
        DDA_HIP_CHECK(hipMemcpyAsync(c->eps_dev.p, eps + 2 * int64_t(e0) * n, cnt * sizeof(z128),
                                     hipMemcpyHostToDevice, c->stream));
        eps_dev = c->eps_dev.as<z128>();
    }
    DDA_HIP_CHECK(hipMemcpyAsync(c->matsys.p, hs.data(), sb, hipMemcpyHostToDevice, c->stream));
    DDA_HIP_CHECK(hipMemsetAsync(err, 0, size_t(ns) * sizeof(int), c->stream));
    if (need128) c->ainv128.ensure(cnt * sizeof(z128));
    if (need64) c->ainv64.ensure(cnt * sizeof(z64));
    dda::MatParams mp{c->opt.polarizability, c->d};
    dda::launch_material(eps_dev, c->matsys.as<dda::MatSys>(), n, ns, mp, nullptr,
                         need128 ? c->ainv128.as<z128>() : nullptr,
                         need64 ? c->ainv64.as<z64>() : nullptr, w_dev, err, c->stream);
    c->host_misc.ensure(size_t(ns) * sizeof(int));
    DDA_HIP_CHECK(hipMemcpyAsync(c->host_misc.p, err, size_t(ns) * sizeof(int),
                                 hipMemcpyDeviceToHost, c->stream));
    wait_stream(c);  // also keeps hs alive until its copy has run
    for (int i = 0; i < ns; ++i) {
        const int herr = c->host_misc.as<int>()[i];
        if (herr == 1) throw Error(DDA_EINVAL, "permittivity is not finite");
        if (herr != 0)
            throw Error(DDA_EINVAL, "permittivity gives a zero or infinite polarizability");
    }
}

// Per-chunk device tables: slot -> system, system -> D pointer.
template <typename T>
const dda::cx<T>* const* upload_dptrs(dda_ctx* c, const std::vector<DEntry*>& ents);
template <>
const z128* const* upload_dptrs<double>(dda_ctx* c, const std::vector<DEntry*>& ents) {
    std::vector<const z128*> h;
    for (auto* e : ents) h.push_back(e->d128.as<z128>());
    c->dptr.ensure(2 * h.size() * sizeof(void*));
    upload(c, c->dptr.p, h.data(), h.size() * sizeof(void*));
    return c->dptr.as<const z128* const>();
}
template <>
const z64* const* upload_dptrs<float>(dda_ctx* c, const std::vector<DEntry*>& ents) {
    std::vector<const z64*> h;
    for (auto* e : ents) h.push_back(e->d64.as<z64>());
    c->dptr.ensure(2 * h.size() * sizeof(void*));
    auto* base = reinterpret_cast<char*>(c->dptr.p) + h.size() * sizeof(void*);
    upload(c, base, h.data(), h.size() * sizeof(void*));
    return reinterpret_cast<const z64* const*>(base);
}


void ensure_slots(dda_ctx* c, int nslots) {
    c->st.ensure(size_t(nslots) * sizeof(dda::BicgSlot));
    c->partial.ensure(size_t(nslots) * c->max_blocks * 8 * sizeof(double));
    c->slot_sys.ensure(size_t(nslots) * sizeof(int));
    c->act.ensure(nslots);
    c->ring.ensure(nslots);
    c->host_st.ensure(size_t(nslots) * sizeof(dda::BicgSlot));
}

void upload_act(dda_ctx* c, const std::vector<int>& act) { c->act.upload(c->stream, act); }

std::vector<dda::BicgSlot> read_states(dda_ctx* c, int nslots) {
    DDA_HIP_CHECK(hipMemcpyAsync(c->host_st.p, c->st.p, size_t(nslots) * sizeof(dda::BicgSlot),
                                 hipMemcpyDeviceToHost, c->stream));
    wait_stream(c);
    auto* p = c->host_st.as<dda::BicgSlot>();
    return std::vector<dda::BicgSlot>(p, p + nslots);
}

// Work vectors of one precision inside a chunk.
template <typename T>
struct Vecs {
    dda::cx<T>*r, *rhat, *p, *v, *s, *t;
};

// BiCGStab over the slots of a chunk, from x0 = 0.  b and x are
// slot-indexed.  The host only looks at the device scalars every
// `check_every` iterations: converged or broken-down slots leave the active
// list; with true_check a slot reporting convergence is verified with a true
// residual b - A x and restarted from it when it drifted above tol.
template <typename T>
void run_bicgstab(dda_ctx* c, int nslots, const dda::cx<T>* b, dda::cx<T>* x, Vecs<T> w,
                  double tol, int maxit, bool true_check, const dda::cx<T>* const* dptr,
                  const dda::cx<T>* ainv, std::vector<int>& iters, std::vector<int>& matvecs,
                  std::vector<int>& status, std::vector<double>& relres) {
    const int64_t nv = c->nv();
    hipStream_t s = c->stream;
    auto* st = c->st.as<dda::BicgSlot>();
    const int* slot_sys = c->slot_sys.as<int>();
    auto red = red_of(c);
    std::vector<int> act(nslots);
    for (int i = 0; i < nslots; ++i) act[i] = i;
    upload_act(c, act);
    const int* dact = c->act.ptr();
    dda::bicg_norm_b<T>(b, st, dact, nslots, nv, tol * tol, 0.0, maxit, red, s);
    DDA_HIP_CHECK(hipMemsetAsync(x, 0, size_t(nslots) * nv * sizeof(dda::cx<T>), s));
    DDA_HIP_CHECK(hipMemcpyAsync(w.r, b, size_t(nslots) * nv * sizeof(dda::cx<T>),
                                 hipMemcpyDeviceToDevice, s));
    dda::bicg_reset<T>(w.r, w.rhat, w.p, w.v, st, dact, nslots, nv, red, s);
    std::vector<int> restarts(nslots, 0);
    status.assign(nslots, DDA_OK);
    iters.assign(nslots, 0);
    matvecs.assign(nslots, 0);
    relres.assign(nslots, 0.0);
    const int check = std::max(1, c->opt.check_every);
    autotune<T>(c, ctx_work(c), dact, nslots, dptr, slot_sys);  // outside any capture
    const bool graphs = use_graphs(c);
    c->graph.drop();
    // One interval of `check` iterations over the n_act slots listed in dact.
    const dda::SlotFilter all{nullptr, dda::FILTER_ALL};
    // For a small batch the p and s updates are folded into the x kernels of
    // v = A p and t = A s (two vector kernels less per iteration; the same
    // p and s bit for bit, ||s||^2 summed over another partition); for a
    // large one the row sums in every block of those kernels cost more than
    // the launches save.
    const int nblk_xr = dda::cocg_rows(nv, red.max_blocks);  // rows of k_update_xr
    auto interval = [&](int n_act) {
        const int nblk_mv = pack_blocks(c, int(sizeof(dda::cx<T>)));
        const int nblk_x = x_blocks(c, int(sizeof(dda::cx<T>)));
        if (nblk_x > red.max_blocks) throw Error(DDA_EDEVICE, "x kernel rows exceed the scratch");
        const bool fold_s = n_act <= kBicgFoldMaxSlots;
        for (int k = 0; k < check; ++k) {
            if (fold_s) {  // p update folded into the x kernel of v = A p
                matvec<T>(c, w.p, w.v, dact, n_act, dptr, slot_sys, ainv, dda::PACK_AX_DOTW, w.r,
                          all, w.rhat, dda::CocgFold{},
                          dda::BicgFold{st, red, dda::BICG_FOLD_P, k > 0 ? nblk_xr : 0, w.v});
            } else {
                dda::bicg_update_p<T>(w.r, w.p, w.v, st, dact, n_act, nv, red, k > 0, s);
                matvec<T>(c, w.p, w.v, dact, n_act, dptr, slot_sys, ainv, dda::PACK_AX_DOTW,
                          nullptr, all, w.rhat);
            }
            if (fold_s) {
                matvec<T>(c, w.s, w.t, dact, n_act, dptr, slot_sys, ainv, dda::PACK_AX_TS, w.r,
                          all, nullptr, dda::CocgFold{},
                          dda::BicgFold{st, red, dda::BICG_FOLD_S, nblk_mv, w.v});
            } else {
                dda::bicg_update_s<T>(w.r, w.v, w.s, st, dact, n_act, nv, red, nblk_mv, s);
                matvec<T>(c, w.s, w.t, dact, n_act, dptr, slot_sys, ainv, dda::PACK_AX_TS);
            }
            dda::bicg_update_xr<T>(x, w.r, w.rhat, w.p, w.s, w.t, st, dact, n_act, nv, red,
                                   nblk_mv, fold_s ? nblk_x : 0, s);
        }
        dda::bicg_finish(st, dact, n_act, nv, red, s);
    };
    try {
        while (true) {
            auto S = read_states(c, nslots);
            std::vector<int> verify, next;
            for (int i : act) {
                iters[i] = S[i].iters;  // device counter, cumulative over restarts
                if (S[i].status == dda::SLOT_CONVERGED || S[i].status == dda::SLOT_BREAKDOWN) {
                    verify.push_back(i);
                } else if (iters[i] >= maxit) {
                    status[i] = DDA_ENOCONV;
                    relres[i] = S[i].bnorm2 > 0 ? std::sqrt(S[i].rnorm2 / S[i].bnorm2) : 0.0;
                } else {
                    next.push_back(i);
                }
            }
            if (!verify.empty() && !true_check) {
                for (int i : verify) {
                    relres[i] = S[i].bnorm2 > 0 ? std::sqrt(S[i].rnorm2 / S[i].bnorm2) : 0.0;
                    status[i] = S[i].status == dda::SLOT_BREAKDOWN ? DDA_EBREAKDOWN : DDA_OK;
                }
            } else if (!verify.empty()) {
                // true residual: y = A x into w.t, r = b - y (rnorm2)
                upload_act(c, verify);
                matvec<T>(c, x, w.t, dact, int(verify.size()), dptr, slot_sys, ainv, dda::PACK_AX);
                dda::residual<T>(b, w.t, w.r, st, dact, int(verify.size()), nv, red, s);
                auto S2 = read_states(c, nslots);
                std::vector<int> again;
                for (int i : verify) {
                    matvecs[i] += 1;
                    const double rr = S2[i].bnorm2 > 0 ? std::sqrt(S2[i].rnorm2 / S2[i].bnorm2) : 0.0;
                    relres[i] = rr;
                    if (rr <= tol) {
                        status[i] = DDA_OK;
                    } else if (restarts[i] >= kMaxRestarts || iters[i] >= maxit) {
                        status[i] = S[i].status == dda::SLOT_BREAKDOWN ? DDA_EBREAKDOWN : DDA_ENOCONV;
                    } else {
                        restarts[i] += 1;
                        again.push_back(i);
                    }
                }
                if (!again.empty()) {
                    upload_act(c, again);
                    dda::bicg_reset<T>(w.r, w.rhat, w.p, w.v, st, dact, int(again.size()), nv, red, s);
                    next.insert(next.end(), again.begin(), again.end());
                }
            }
            std::sort(next.begin(), next.end());
            act = next;
            const int n_act = int(act.size());
            if (n_act == 0) break;
            upload_act(c, act);
            if (graphs) launch_captured(c, c->graph, n_act, [&] { interval(n_act); });
            else interval(n_act);
            for (int i : act) matvecs[i] += 2 * check;
        }
    } catch (...) {
        (void)hipStreamSynchronize(c->stream);
        c->graph.drop();
        throw;
    }
    c->graph.drop();  // the graph holds this call's buffer addresses
}

// Writes rnorm2 = rn[i]^2 into the device scalars of every slot.
void set_rnorm2(dda_ctx* c, int nslots, const std::vector<double>& rn) {
    auto S = read_states(c, nslots);
    for (int i = 0; i < nslots; ++i) S[i].rnorm2 = rn[i] * rn[i];
    std::memcpy(c->host_st.p, S.data(), S.size() * sizeof(dda::BicgSlot));
    DDA_HIP_CHECK(hipMemcpyAsync(c->st.p, c->host_st.p, S.size() * sizeof(dda::BicgSlot),
                                 hipMemcpyHostToDevice, c->stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
}

// Mixed precision: x = 0, r = b; repeat { d = FP32-BiCGStab(A, r/||r||) to
// kInnerTol; x += ||r|| d; r = b - A x in FP64 } until ||r|| <= tol ||b||.
void run_mixed(dda_ctx* c, int nslots, const z128* b, z128* x, const z128* const* dptr64,
               const z64* const* dptr32, std::vector<int>& iters, std::vector<int>& mvs,
               std::vector<int>& status, std::vector<double>& relres) {
    const int64_t nv = c->nv();
    const size_t q = size_t(nslots) * nv;
    c->vec128.ensure(2 * q * sizeof(z128));
    c->vec64.ensure(8 * q * sizeof(z64));
    auto* V = c->vec128.as<z128>();
    auto* U = c->vec64.as<z64>();
    z128* r64 = V;
    z128* y64 = V + q;
    z64* r32 = U;
    z64* d32 = U + q;
    Vecs<float> w{U + 2 * q, U + 3 * q, U + 4 * q, U + 5 * q, U + 6 * q, U + 7 * q};
    auto* st = c->st.as<dda::BicgSlot>();
    auto red = red_of(c);
    const double tol = c->opt.tol;
    iters.assign(nslots, 0);
    mvs.assign(nslots, 0);
    status.assign(nslots, DDA_ENOCONV);
    relres.assign(nslots, 1.0);
    std::vector<int> all(nslots);
    for (int i = 0; i < nslots; ++i) all[i] = i;
    upload_act(c, all);
    dda::bicg_norm_b<double>(b, st, c->act.ptr(), nslots, nv, tol * tol, 0.0, c->opt.maxit,
                             red, c->stream);
    std::vector<double> bn(nslots), rn(nslots);
    {
        auto S = read_states(c, nslots);
        for (int i = 0; i < nslots; ++i) bn[i] = rn[i] = std::sqrt(S[i].bnorm2);
    }
    DDA_HIP_CHECK(hipMemsetAsync(x, 0, q * sizeof(z128), c->stream));
    DDA_HIP_CHECK(hipMemcpyAsync(r64, b, q * sizeof(z128), hipMemcpyDeviceToDevice, c->stream));
    std::vector<int> stalls(nslots, 0);
    for (int outer = 0; outer < kMaxOuter; ++outer) {
        std::vector<int> need;
        std::vector<char> isneed(nslots, 0);
        for (int i = 0; i < nslots; ++i) {
            relres[i] = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
            if (relres[i] <= tol) status[i] = DDA_OK;
            else if (iters[i] < c->opt.maxit && stalls[i] < 3) { need.push_back(i); isneed[i] = 1; }
        }
        if (need.empty()) break;
        // inner right-hand side r/||r|| on the slots that need work, 0 elsewhere
        // (a zero right-hand side converges at once, with no iteration)
        set_rnorm2(c, nslots, rn);
        upload_act(c, need);
        dda::scale_down(r64, r32, st, c->act.ptr(), int(need.size()), nv, c->stream);
        for (int i = 0; i < nslots; ++i)
            if (!isneed[i])
                DDA_HIP_CHECK(hipMemsetAsync(r32 + size_t(i) * nv, 0, nv * sizeof(z64), c->stream));
        std::vector<int> it_in, mv_in, st_in;
        std::vector<double> rr_in;
        run_bicgstab<float>(c, nslots, r32, d32, w, kInnerTol, c->opt.maxit, false, dptr32,
                            c->ainv64.as<z64>(), it_in, mv_in, st_in, rr_in);
        set_rnorm2(c, nslots, rn);
        upload_act(c, need);
        dda::accumulate_up(x, d32, st, c->act.ptr(), int(need.size()), nv, c->stream);
        matvec<double>(c, x, y64, c->act.ptr(), int(need.size()), dptr64,
                       c->slot_sys.as<int>(), c->ainv128.as<z128>(), dda::PACK_AX);
        dda::residual<double>(b, y64, r64, st, c->act.ptr(), int(need.size()), nv, red,
                              c->stream);
        auto S = read_states(c, nslots);
        for (int i : need) {
            iters[i] += it_in[i];
            mvs[i] += mv_in[i] + 1;
            const double nr = std::sqrt(S[i].rnorm2);
            stalls[i] = (nr < 0.9 * rn[i]) ? 0 : stalls[i] + 1;
            rn[i] = nr;
        }
    }
    for (int i = 0; i < nslots; ++i) {
        relres[i] = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
        status[i] = relres[i] <= tol ? DDA_OK : DDA_ENOCONV;
    }
}

// COCG (conjugate-orthogonal CG: CG with the bilinear product x^T y, for
// the complex-symmetric DDA matrix), from x0 = 0.  b and x are FP64 and
// slot-indexed; r, p, q are in T.  One matvec per iteration; the direction
// update and p^T q are fused into the matvec.  For T = float the steps
// accumulate in x_lo (FP32) and a reliable update (x += x_lo, r = b - A x in
// FP64, rho from the new r) is made whenever the recursive residual fell by
// kUpdateDrop since the last one, and whenever it reports convergence; for
// T = double only the convergence is verified that way.
//
// The device drives the iteration.  Work goes out in intervals: a check
// phase (the FP64 residual of every slot that asked for one decides
// convergence, the iteration limit, a restart after a breakdown or a reliable
// update) followed by check_every iterations of the slots still iterating;
// every kernel skips the slots its filter rejects.  The host never waits
// inside an interval: after each one the slot states are copied to pinned
// memory, and before sending interval k the host reads the copy made after
// interval k - kLag (already complete while interval k - 1 runs) and drops the
// finished slots from the active list.  On a non-default stream an interval
// is a captured graph, replayed while the active list keeps its length.
constexpr double kUpdateDrop = 0.1;
constexpr int kLag = 2;

// Buffers of one COCG driver (a dda_solve chunk, or an engine's slot pool).
template <typename T>
struct CocgBufs {
    Work w;
    const int* act;       // device active list
    const int* slot_sys;  // slot -> system (D and 1/alpha row)
    const z128* b;
    z128* x;
    dda::cx<T>*r, *p, *q;
    z64* x_lo;  // FP32 step accumulator (T = float)
    z128* y64;  // FP64 matvec output of the check phase
    const dda::cx<T>* const* dptr;
    const dda::cx<T>* ainv;
    const z128* const* dptr64;
    const z128* ainv64;
    // QMR (solver DDA_SOLVER_QMR): r holds u = A v_n (and the check's
    // residual), p and q the Lanczos vectors, pa and pb the directions
    dda::cx<T>* pa = nullptr;
    dda::cx<T>* pb = nullptr;
    bool qmr = false;
};

// x = 0, r = b, scalars for the n listed slots (device list act).
template <typename T>
void cocg_init(dda_ctx* c, const CocgBufs<T>& B, const int* act, int n, double tol, int maxit) {
    constexpr bool mixed = std::is_same<T, float>::value;
    const int64_t nv = c->nv();
    dda::bicg_norm_b<double>(B.b, B.w.st, act, n, nv, tol * tol,
                             mixed && !B.qmr ? kUpdateDrop * kUpdateDrop : 0.0, maxit, B.w.red,
                             c->stream);
    dda::cocg_zero(B.x, mixed ? B.x_lo : nullptr, act, n, nv, c->stream);
    dda::cocg_start<T>(B.b, nullptr, B.r, B.w.st, act, n, nv, B.w.red, c->stream);
}

// One interval over the n_act slots of B.act.
template <typename T>
void cocg_interval(dda_ctx* c, const CocgBufs<T>& B, int n_act) {
    constexpr bool mixed = std::is_same<T, float>::value;
    const int64_t nv = c->nv();
    hipStream_t s = c->stream;
    const dda::SlotFilter fchk{B.w.st, dda::FILTER_CHECK}, fact{B.w.st, dda::FILTER_ACTIVE};
    auto* xs = mixed ? reinterpret_cast<dda::cx<T>*>(B.x_lo) : reinterpret_cast<dda::cx<T>*>(B.x);
    if (mixed) dda::accumulate_lo(B.x, B.x_lo, B.act, n_act, nv, fchk, s);
    matvec<double>(c, B.w, B.x, B.y64, B.act, n_act, B.dptr64, B.slot_sys, B.ainv64, dda::PACK_AX,
                   nullptr, fchk);
    dda::cocg_check<T>(B.b, B.y64, B.r, B.w.st, B.act, n_act, nv, kMaxRestarts, B.w.red, s,
                       B.qmr);
    if (B.qmr) {
        // a cycle starts from the residual of every slot the check left
        // iterating; an even number of steps brings the roles of the vectors
        // and of the scalar copies back to where the next interval expects them
        dda::qmr_start<T>(B.r, B.p, B.q, B.pa, B.pb, B.w.st, B.act, n_act, nv,
                          mixed ? kQmrInner : 0.0, s);
        const int steps = std::max(2, (c->opt.check_every + 1) / 2 * 2);
        const int nblk = pack_blocks(c, int(sizeof(dda::cx<T>)));
        for (int k = 0; k < steps; ++k) {
            const int par = k & 1;
            dda::cx<T>* vc = par ? B.q : B.p;
            dda::cx<T>* vo = par ? B.p : B.q;
            dda::cx<T>* p1 = par ? B.pa : B.pb;
            dda::cx<T>* p2 = par ? B.pb : B.pa;
            matvec<T>(c, B.w, vc, B.r, B.act, n_act, B.dptr, B.slot_sys, B.ainv,
                      dda::PACK_AX_COCG, nullptr, fact);
            dda::qmr_step<T>(xs, B.r, vc, vo, p1, p2, B.w.st, B.act, n_act, nv, B.w.red, nblk,
                             par, s);
        }
        return;
    }
    // For a small batch, where an iteration's time is the latency of its
    // kernels, the end of each iteration but the last is folded into the
    // next one's direction update (one kernel less per iteration; rho
    // alternates between two copies so that no block of that kernel reads a
    // value another block writes).  For a large batch the row sums it adds to
    // every block of the x kernel cost more than the launch it saves.  Either
    // way the arithmetic is the same, bit for bit.
    const int check = std::max(1, c->opt.check_every);
    const int rows = dda::cocg_rows(nv, B.w.red.max_blocks);
    const bool fold_fin = n_act <= kCocgFoldMaxSlots;
    for (int k = 0; k < check; ++k) {
        const dda::CocgFold fold = (k == 0 || !fold_fin)
                                       ? dda::CocgFold{}
                                       : dda::CocgFold{B.w.st, B.w.red, rows, (k - 1) & 1};
        matvec<T>(c, B.w, B.p, B.q, B.act, n_act, B.dptr, B.slot_sys, B.ainv, dda::PACK_AX_COCG,
                  B.r, fact, nullptr, fold);
        const bool last = !fold_fin || k == check - 1;
        dda::cocg_update_xr<T>(xs, B.r, B.p, B.q, B.w.st, B.act, n_act, nv, B.w.red,
                               pack_blocks(c, int(sizeof(dda::cx<T>))), fold_fin ? (k & 1) : 0,
                               last, s);
    }
}

int status_of(int slot_status) {
    switch (slot_status) {
        case dda::SLOT_DONE: return DDA_OK;
        case dda::SLOT_FAIL_NOCONV: return DDA_ENOCONV;
        case dda::SLOT_FAIL_BREAKDOWN: return DDA_EBREAKDOWN;
        case dda::SLOT_FAIL_INVALID: return DDA_EINVAL;
        default: throw Error(DDA_EDEVICE, "COCG slot left in a non-terminal state");
    }
}

dda_solve_info info_of(const dda::BicgSlot& S) {
    const double rr = S.bnorm2 > 0 ? std::sqrt(S.rnorm2 / S.bnorm2) : 0.0;
    return dda_solve_info{S.iters, S.matvecs, rr, status_of(S.status)};
}

// Solves every slot of a dda_solve chunk.
template <typename T>
void run_cocg(dda_ctx* c, int nslots, const CocgBufs<T>& B, double tol, int maxit,
              std::vector<dda_solve_info>& info) {
    std::vector<int> act(nslots);
    for (int i = 0; i < nslots; ++i) act[i] = i;
    upload_act(c, act);
    cocg_init<T>(c, B, B.act, nslots, tol, maxit);
    autotune<T>(c, B.w, B.act, nslots, B.dptr, B.slot_sys);  // outside any capture
    autotune<double>(c, B.w, B.act, nslots, B.dptr64, B.slot_sys);
    const bool graphs = use_graphs(c);
    c->graph.drop();
    try {
        for (int64_t k = 0;; ++k) {
            if (k >= kLag) {
                const dda::BicgSlot* S = c->ring.wait(k - kLag);
                std::vector<int> next;
                next.reserve(act.size());
                for (int i : act)
                    if (!dda::slot_terminal(S[i].status)) next.push_back(i);
                if (next.empty()) break;
                if (next.size() != act.size()) {
                    act.swap(next);
                    upload_act(c, act);
                }
            }
            const int n_act = int(act.size());
            if (graphs) launch_captured(c, c->graph, n_act, [&] { cocg_interval<T>(c, B, n_act); });
            else cocg_interval<T>(c, B, n_act);
            c->ring.snapshot(c->stream, B.w.st, nslots, k);
        }
    } catch (...) {
        (void)hipStreamSynchronize(c->stream);
        c->graph.drop();
        throw;
    }
    c->graph.drop();  // the graph holds this chunk's buffer addresses
    auto S = read_states(c, nslots);
    info.resize(nslots);
    for (int i = 0; i < nslots; ++i) info[i] = info_of(S[i]);
}

// Sizes of the per-slot work space, in bytes.
size_t slot_bytes(const dda_ctx* c, bool mixed) {
    const size_t ge = size_t(dda::grid_elems(c->g));
    const size_t nv = size_t(c->nv());
    const size_t red = size_t(c->max_blocks) * 8 * sizeof(double) + sizeof(dda::BicgSlot);
    // BiCGStab: six vectors (FP64), or two FP64 and eight FP32 (mixed); COCG
    // and QMR (six vectors at most) fit in the same
    if (!mixed) return ge * sizeof(z128) + 6 * nv * sizeof(z128) + red;
    return ge * sizeof(z128) + 2 * nv * sizeof(z128) + 8 * nv * sizeof(z64) + red;
}

void host_trajectory_check(const dda_ctx* c, const double* r0, int n_traj) {
    const dda::Geo& g = c->g;
    for (int t = 0; t < n_traj; ++t) {
        for (int q = 0; q < 3; ++q) check_finite(r0[3 * t + q], "trajectory coordinate");
        for (int iy = 0; iy < g.ny; ++iy)
            for (int ix = 0; ix < g.nx; ++ix) {
                if (!c->occ_col[size_t(iy) * g.nx + ix]) continue;
                const double px = c->d * (ix - 0.5 * g.nx + 0.5);
                const double py = c->d * (iy - 0.5 * g.ny + 0.5);
                if (std::hypot(px - r0[3 * t], py - r0[3 * t + 1]) < 1e-9 * c->d)
                    throw Error(DDA_ESINGULAR,
                                "trajectory passes through a dipole centre (b = 0 in eq. 25)");
            }
    }
}

void check_energies(int n_energy, const double* energy) {
    if (n_energy < 0) throw Error(DDA_EINVAL, "n_energy < 0");
    for (int e = 0; e < n_energy; ++e) {
        check_finite(energy[e], "energy");
        if (energy[e] <= 0) throw Error(DDA_EINVAL, "energies must be positive");
    }
}

void check_beta(dda_ctx* c, double beta) {
    check_finite(beta, "beta");
    if (!(beta > 0.0 && beta < 1.0)) throw Error(DDA_EINVAL, "beta must lie in (0, 1)");
    (void)gamma_h_of(beta, c->mh);
}

// Number of systems per chunk that fit the work-space budget.
int systems_per_chunk(dda_ctx* c, int n_energy, int n_traj, bool mixed) {
    size_t free_b = 0, total_b = 0;
    DDA_HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    const size_t dsz = d_elems(c, 16) * sizeof(z128) + (mixed ? d_elems(c, 8) * sizeof(z64) : 0);
    const size_t per_sys = size_t(n_traj) * slot_bytes(c, mixed) + dsz +
                           size_t(c->g.n_occ) * (sizeof(z128) + sizeof(z64));
    const size_t budget = std::min<size_t>(free_b / 10 * 7, size_t(96) << 30);
    int ns = int(std::max<size_t>(1, budget / std::max<size_t>(per_sys, 1)));
    ns = std::min(ns, n_energy);
    ns = std::min(ns, std::max(1, 65535 / std::max(1, n_traj)));
    return std::max(ns, 1);
}

}  // namespace


// ==================================================== continuous batching
// A slot pool over one lattice.  Systems (one energy, one right-hand side)
// are submitted at any time; between intervals the engine admits queued
// systems into free slots (material terms, D from the context's cache,
// initial state), runs the same device-driven COCG intervals as dda_solve
// over every occupied slot, and harvests the slots whose lagged state
// snapshot shows them finished (final iterate copied to the caller's buffer,
// slot freed).  All its buffers are its own, so other calls on the context
// (dda_eels_cl for finished requests) may run between polls.
struct Pending {
    int64_t tag;
    double energy;
    cplx mh;  // host index of the lattice's context when the system was submitted
    std::vector<double> eps;  // [n][2]
    const z128* einc;         // [3][n]
    z128* out;                // [3][n]
    const dda_ctx* lat;       // the system's lattice (its index map, n dipoles)
};

struct SlotRec {
    bool busy = false;
    int64_t tag = 0;
    int64_t admitted = 0;  // first interval the system takes part in
    DEntry* d = nullptr;
    z128* out = nullptr;
    const dda_ctx* lat = nullptr;
};

struct Engine {
    int cap = 0;
    bool mixed = false;
    DevBuf st, partial, slot_sys, G, b, x, r, p, q, xlo, y64, ainv128, ainv64, dtab, eps, msys, err;
    DevBuf maps;                     // [cap][nx ny nz]: each slot's lattice index map
    PinnedBuf h_eps, h_small;        // staging of admitted permittivities and tables
    hipEvent_t stage_ev = nullptr;   // the last copy out of the staging buffers
    hipEvent_t out_ev = nullptr;     // a harvest copy, for the stream of another lattice
    ActRing act, adm;                // interval list; list of slots being admitted
    StateRing ring;
    GraphCache graph;
    std::vector<SlotRec> slots;
    std::vector<const void*> dtab_h;  // [2][cap]: FP64 D pointers, then FP32
    std::vector<int> running;         // occupied slots, sorted
    bool act_dirty = true;
    std::deque<Pending> queue;
    std::mutex mu;  // guards queue: dda_engine_submit may run on another thread
    int64_t sent = 0;  // intervals sent
    std::deque<std::pair<int64_t, dda_solve_info>> done;
    // sizes of running and done as the polling thread last left them, for
    // dda_engine_status from other threads
    std::atomic<int> n_running{0}, n_done{0};
    void publish() {
        n_running.store(int(running.size()), std::memory_order_relaxed);
        n_done.store(int(done.size()), std::memory_order_relaxed);
    }
    Engine() = default;
    Engine(const Engine&) = delete;
    ~Engine() {
        if (stage_ev) (void)hipEventDestroy(stage_ev);
        if (out_ev) (void)hipEventDestroy(out_ev);
    }
};

namespace {

// Device bytes of one engine slot, counting the D of a distinct energy.
size_t engine_slot_bytes(const dda_ctx* c, bool mixed) {
    const size_t nv = size_t(c->nv()), n = size_t(c->g.n_occ);
    const size_t ge = size_t(dda::grid_elems(c->g));
    size_t b = 3 * nv * sizeof(z128);                                   // b, x, y64
    b += mixed ? 4 * nv * sizeof(z64) : 3 * nv * sizeof(z128);          // r, p, q (x_lo)
    b += n * (sizeof(z128) + (mixed ? sizeof(z64) : 0));                // 1/alpha
    b += n * sizeof(z128);                                              // eps staging
    b += ge * sizeof(z128);                                             // grid work buffer
    b += size_t(c->g.nx) * c->g.ny * c->g.nz * sizeof(int);            // index map
    b += size_t(c->max_blocks) * 8 * sizeof(double) + sizeof(dda::BicgSlot) + 64;
    b += d_elems(c, 16) * sizeof(z128) + (mixed ? d_elems(c, 8) * sizeof(z64) : 0);
    return b;
}

template <typename T>
CocgBufs<T> engine_bufs(dda_ctx* c, Engine& E, const int* act) {
    const size_t nv = size_t(c->nv());
    const int64_t cells = int64_t(c->g.nx) * c->g.ny * c->g.nz;
    const Work w{E.st.as<dda::BicgSlot>(), dda::RedScratch{E.partial.as<double>(), c->max_blocks},
                 E.G.p, E.maps.as<int>(), cells};
    auto** tab = reinterpret_cast<const void**>(E.dtab.p);
    constexpr bool mixed = std::is_same<T, float>::value;
    CocgBufs<T> B{w, act, E.slot_sys.as<int>(), E.b.as<z128>(), E.x.as<z128>(),
                  nullptr, nullptr, nullptr, mixed ? E.xlo.as<z64>() : nullptr, E.y64.as<z128>(),
                  nullptr, nullptr,
                  reinterpret_cast<const z128* const*>(tab), E.ainv128.as<z128>()};
    auto* R = static_cast<dda::cx<T>*>(E.r.p);
    B.r = R;
    B.p = R + nv * E.cap;
    B.q = R + 2 * nv * E.cap;
    if constexpr (mixed) {
        B.dptr = reinterpret_cast<const z64* const*>(tab + E.cap);
        B.ainv = E.ainv64.as<z64>();
    } else {
        B.dptr = reinterpret_cast<const z128* const*>(tab);
        B.ainv = E.ainv128.as<z128>();
    }
    return B;
}

void engine_open(dda_ctx* c, int cap) {
    if (c->opt.solver != DDA_SOLVER_COCG)
        throw Error(DDA_EINVAL, "the batching engine runs the COCG solver");
    if (c->g.n_occ == 0) throw Error(DDA_EINVAL, "the lattice has no dipoles");
    if (cap < 1 || cap > 4096) throw Error(DDA_EINVAL, "max_slots must lie in [1, 4096]");
    auto E = std::make_unique<Engine>();
    E->cap = cap;
    E->mixed = c->opt.precision == DDA_PREC_MIXED;
    // D entries beyond one per slot (dda_workspace_bytes counts those) are
    // evicted, their buffers reused by the next wavenumber
    c->dcache_limit = std::min(c->dcache_limit,
                               size_t(cap) * (d_elems(c, 16) * sizeof(z128) +
                                              (E->mixed ? d_elems(c, 8) * sizeof(z64) : 0)));
    const size_t nv = size_t(c->nv()), n = size_t(c->g.n_occ), k = size_t(cap);
    E->st.ensure(k * sizeof(dda::BicgSlot));
    E->partial.ensure(k * c->max_blocks * 8 * sizeof(double));
    E->slot_sys.ensure(k * sizeof(int));
    E->G.ensure(k * size_t(dda::grid_elems(c->g)) * sizeof(z128));
    E->b.ensure(k * nv * sizeof(z128));
    E->x.ensure(k * nv * sizeof(z128));
    E->y64.ensure(k * nv * sizeof(z128));
    E->r.ensure(3 * k * nv * (E->mixed ? sizeof(z64) : sizeof(z128)));
    if (E->mixed) E->xlo.ensure(k * nv * sizeof(z64));
    E->ainv128.ensure(k * n * sizeof(z128));
    if (E->mixed) E->ainv64.ensure(k * n * sizeof(z64));
    E->dtab.ensure(2 * k * sizeof(void*));
    E->eps.ensure(k * n * sizeof(z128));
    E->msys.ensure(k * sizeof(dda::MatSys));
    E->err.ensure(k * sizeof(int));
    E->h_eps.ensure(k * n * sizeof(z128));
    E->h_small.ensure(k * (sizeof(dda::MatSys) + 2 * sizeof(void*)));
    E->maps.ensure(k * size_t(c->g.nx) * c->g.ny * c->g.nz * sizeof(int));
    DDA_HIP_CHECK(hipEventCreateWithFlags(&E->stage_ev, hipEventDisableTiming));
    DDA_HIP_CHECK(hipEventCreateWithFlags(&E->out_ev, hipEventDisableTiming));
    E->act.ensure(cap);
    E->adm.ensure(cap);
    E->ring.ensure(cap);
    E->slots.resize(cap);
    E->dtab_h.assign(2 * k, nullptr);
    std::vector<int> ident(cap);
    for (int i = 0; i < cap; ++i) ident[i] = i;
    upload(c, E->slot_sys.p, ident.data(), k * sizeof(int));
    // slot states start terminal: a snapshot of a never-used slot reads as free
    std::vector<dda::BicgSlot> init(cap);
    for (auto& S : init) {
        std::memset(&S, 0, sizeof(S));
        S.status = dda::SLOT_DONE;
    }
    upload(c, E->st.p, init.data(), k * sizeof(dda::BicgSlot));
    c->engine = std::move(E);
}

void engine_release(dda_ctx* c, SlotRec& sr) {
    if (sr.d) sr.d->refs -= 1;
    sr = SlotRec{};
    (void)c;
}

// Slots whose snapshot after interval j shows them finished.
void engine_harvest(dda_ctx* c, Engine& E, int64_t j) {
    const dda::BicgSlot* S = E.ring.wait(j);
    const size_t nv = size_t(c->nv());
    std::vector<int> keep;
    keep.reserve(E.running.size());
    for (int s : E.running) {
        SlotRec& sr = E.slots[s];
        if (sr.admitted <= j && dda::slot_terminal(S[s].status)) {
            const size_t n = size_t(sr.lat->g.n_occ), cap_n = size_t(c->g.n_occ);
            // [3][n] out of the slot's [3][cap_n]
            DDA_HIP_CHECK(hipMemcpy2DAsync(sr.out, n * sizeof(z128),
                                           E.x.as<z128>() + size_t(s) * nv, cap_n * sizeof(z128),
                                           n * sizeof(z128), 3, hipMemcpyDeviceToDevice,
                                           c->stream));
            if (sr.lat != c) {  // the lattice's own stream reads the result next
                DDA_HIP_CHECK(hipEventRecord(E.out_ev, c->stream));
                DDA_HIP_CHECK(hipStreamWaitEvent(sr.lat->stream, E.out_ev, 0));
            }
            E.done.emplace_back(sr.tag, info_of(S[s]));
            engine_release(c, sr);
        } else {
            keep.push_back(s);
        }
    }
    if (keep.size() != E.running.size()) {
        E.running.swap(keep);
        E.publish();
        E.act_dirty = true;
    }
}

// Zeroes every per-slot vector of slot s (outside any capture): a matvec
// writes only the entries of the slot's dipoles, so the entries past them
// must start, and then stay, zero.
template <typename T>
void engine_clear_slot(dda_ctx* c, Engine& E, int s) {
    const size_t nv = size_t(c->nv()), cap = size_t(E.cap);
    hipStream_t st = c->stream;
    for (DevBuf* v : {&E.b, &E.x, &E.y64})
        DDA_HIP_CHECK(hipMemsetAsync(v->as<z128>() + size_t(s) * nv, 0, nv * sizeof(z128), st));
    auto* R = static_cast<dda::cx<T>*>(E.r.p);
    for (int j = 0; j < 3; ++j)
        DDA_HIP_CHECK(hipMemsetAsync(R + j * nv * cap + size_t(s) * nv, 0,
                                     nv * sizeof(dda::cx<T>), st));
    if (E.xlo.p)
        DDA_HIP_CHECK(hipMemsetAsync(E.xlo.as<z64>() + size_t(s) * nv, 0, nv * sizeof(z64), st));
}

template <typename T>
void engine_admit(dda_ctx* c, Engine& E) {
    constexpr bool mixed = std::is_same<T, float>::value;
    std::vector<int> free_slots;
    for (int s = 0; s < E.cap; ++s)
        if (!E.slots[s].busy) free_slots.push_back(s);
    std::vector<Pending> take;
    {
        std::lock_guard<std::mutex> lk(E.mu);
        while (!E.queue.empty() && take.size() < free_slots.size()) {
            take.push_back(std::move(E.queue.front()));
            E.queue.pop_front();
        }
    }
    if (take.empty()) return;
    const int na = int(take.size());
    const size_t n = size_t(c->g.n_occ), nv = size_t(c->nv());
    const int64_t cells = int64_t(c->g.nx) * c->g.ny * c->g.nz;
    wait_event(E.stage_ev);  // the previous admission's copies have run
    auto* heps = E.h_eps.as<double>();
    auto* hsys = E.h_small.as<dda::MatSys>();
    auto** htab = reinterpret_cast<const void**>(hsys + E.cap);
    std::vector<int> adm(na);
    c->pin_clock = c->use_clock + 1;
    for (int i = 0; i < na; ++i) {
        const int s = free_slots[i];
        adm[i] = s;
        Pending& pd = take[i];
        DEntry* d = get_D_k(c, pd.mh * (pd.energy / kHbarC), mixed);
        d->refs += 1;
        SlotRec& sr = E.slots[s];
        sr.busy = true;
        sr.tag = pd.tag;
        sr.admitted = E.sent;
        sr.d = d;
        sr.out = pd.out;
        sr.lat = pd.lat;
        E.dtab_h[s] = d->d128.p;
        E.dtab_h[E.cap + s] = mixed ? d->d64.p : nullptr;
        const size_t ns = size_t(pd.lat->g.n_occ);
        // a lattice with fewer dipoles than the slot holds fills a prefix;
        // the padding takes its first permittivity (a finite 1/alpha that no
        // matvec reads)
        double* he = heps + 2 * n * size_t(i);
        std::memcpy(he, pd.eps.data(), ns * sizeof(z128));
        for (size_t t = ns; t < n; ++t) {
            he[2 * t] = pd.eps[0];
            he[2 * t + 1] = pd.eps[1];
        }
        const cplx k = pd.mh * (pd.energy / kHbarC);
        hsys[i] = dda::MatSys{k.real(), k.imag(), pd.mh.real(), pd.mh.imag()};
        DDA_HIP_CHECK(hipMemcpyAsync(E.maps.as<int>() + size_t(s) * cells, pd.lat->map.p,
                                     size_t(cells) * sizeof(int), hipMemcpyDeviceToDevice,
                                     c->stream));
        if (ns < n) engine_clear_slot<T>(c, E, s);  // padding entries stay zero in every vector
        DDA_HIP_CHECK(hipMemcpy2DAsync(E.b.as<z128>() + size_t(s) * nv, n * sizeof(z128), pd.einc,
                                       ns * sizeof(z128), ns * sizeof(z128), 3,
                                       hipMemcpyDeviceToDevice, c->stream));
    }
    std::memcpy(htab, E.dtab_h.data(), E.dtab_h.size() * sizeof(void*));
    hipStream_t st = c->stream;
    DDA_HIP_CHECK(hipMemcpyAsync(E.eps.p, heps, size_t(na) * n * sizeof(z128),
                                 hipMemcpyHostToDevice, st));
    DDA_HIP_CHECK(hipMemcpyAsync(E.msys.p, hsys, size_t(na) * sizeof(dda::MatSys),
                                 hipMemcpyHostToDevice, st));
    DDA_HIP_CHECK(hipMemcpyAsync(E.dtab.p, htab, E.dtab_h.size() * sizeof(void*),
                                 hipMemcpyHostToDevice, st));
    DDA_HIP_CHECK(hipEventRecord(E.stage_ev, st));
    E.adm.upload(st, adm);
    DDA_HIP_CHECK(hipMemsetAsync(E.err.p, 0, size_t(na) * sizeof(int), st));
    const dda::MatParams mp{c->opt.polarizability, c->d};
    dda::launch_material(E.eps.as<z128>(), E.msys.as<dda::MatSys>(), int64_t(n), na, mp,
                         E.adm.ptr(), E.ainv128.as<z128>(), mixed ? E.ainv64.as<z64>() : nullptr,
                         nullptr, E.err.as<int>(), st);
    const auto B = engine_bufs<T>(c, E, E.adm.ptr());
    cocg_init<T>(c, B, E.adm.ptr(), na, c->opt.tol, c->opt.maxit);
    dda::mark_invalid(B.w.st, E.adm.ptr(), E.err.as<int>(), na, st);
    E.running.insert(E.running.end(), adm.begin(), adm.end());
    std::sort(E.running.begin(), E.running.end());
    E.publish();
    E.act_dirty = true;
}

template <typename T>
void engine_poll(dda_ctx* c, Engine& E, int max_intervals) {
    const auto B = engine_bufs<T>(c, E, E.act.ptr());
    const bool graphs = use_graphs(c);
    for (int it = 0; it < max_intervals; ++it) {
        if (E.sent >= kLag && !E.running.empty()) engine_harvest(c, E, E.sent - kLag);
        engine_admit<T>(c, E);
        if (E.running.empty()) break;
        if (E.act_dirty) {
            E.act.upload(c->stream, E.running);
            E.act_dirty = false;
        }
        const int n_act = int(E.running.size());
        autotune<T>(c, B.w, B.act, n_act, B.dptr, B.slot_sys);  // once, outside any capture
        autotune<double>(c, B.w, B.act, n_act, B.dptr64, B.slot_sys);
        if (graphs) launch_captured(c, E.graph, n_act, [&] { cocg_interval<T>(c, B, n_act); });
        else cocg_interval<T>(c, B, n_act);
        E.ring.snapshot(c->stream, B.w.st, E.cap, E.sent);
        E.sent += 1;
    }
}

}  // namespace

// ====================================================================== ABI

#define DDA_API_BEGIN try {
#define DDA_API_END                                    \
    }                                                  \
    catch (const dda::Error& e) {                      \
        g_last_error = e.what();                       \
        return e.status;                               \
    }                                                  \
    catch (const std::bad_alloc&) {                    \
        g_last_error = "host allocation failed";       \
        return DDA_ENOMEM;                             \
    }                                                  \
    catch (const std::exception& e) {                  \
        g_last_error = e.what();                       \
        return DDA_EDEVICE;                            \
    }

extern "C" {

void dda_default_options(dda_options* opt) {
    if (!opt) return;
    opt->polarizability = DDA_POL_LDR;
    opt->solver = DDA_SOLVER_BICGSTAB;
    opt->precision = DDA_PREC_FP64;
    opt->tol = 1e-10;
    opt->maxit = 100000;
    opt->check_every = 16;
    opt->use_graphs = 1;
    opt->interaction = DDA_INT_POINT;
}

double dda_beta_from_keV(double kinetic_keV) {
    const double gam = 1.0 + kinetic_keV / kMeC2;
    return std::sqrt(1.0 - 1.0 / (gam * gam));
}

const char* dda_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------- far-field CL -----

int dda_cl_directions(dda_ctx* c, int n_energy, const double* energy_eV, double beta,
                      int n_traj, const void* p_dev, int n_dir, const double* dir_xyz,
                      const double* weight, double* dp_domega, double* p_cl) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (n_energy < 0 || n_traj < 0 || n_dir < 0) throw Error(DDA_EINVAL, "negative size");
    const int64_t nrhs = int64_t(n_energy) * n_traj;
    if (nrhs == 0 || n_dir == 0) return DDA_OK;
    if (!energy_eV || !p_dev || !dir_xyz) throw Error(DDA_EINVAL, "NULL argument");
    if (p_cl && !weight) throw Error(DDA_EINVAL, "p_cl needs the direction weights");
    if (c->mh.imag() != 0.0)
        throw Error(DDA_EINVAL, "far-field CL needs a non-absorbing host (section 2.6)");
    check_energies(n_energy, energy_eV);
    check_beta(c, beta);
    for (int q = 0; q < n_dir; ++q) {
        const double* n = dir_xyz + 3 * q;
        const double r2 = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
        if (!std::isfinite(r2) || std::abs(r2 - 1.0) > 1e-9)
            throw Error(DDA_EINVAL, "directions must be unit vectors");
        if (weight) check_finite(weight[q], "weight");
    }
    const dda::Geo& g = c->g;
    if (g.n_occ == 0) {
        if (dp_domega) std::fill(dp_domega, dp_domega + nrhs * n_dir, 0.0);
        if (p_cl) std::fill(p_cl, p_cl + nrhs, 0.0);
        return DDA_OK;
    }
    if (dda::ff_lds_bytes(g.nx, g.ny, g.nz) > (size_t(64) << 10))
        throw Error(DDA_EINVAL, "lattice sides too long for the far-field phase tables");
    if (!c->ff_coord.p) {
        std::vector<int> pc(c->occ_lin.size());
        for (size_t j = 0; j < pc.size(); ++j) {
            const int lin = c->occ_lin[j];
            const int ix = lin % g.nx, iy = (lin / g.nx) % g.ny, iz = lin / (g.nx * g.ny);
            pc[j] = ix | (iy << 10) | (iz << 20);
        }
        c->ff_coord.ensure(pc.size() * sizeof(int));
        upload(c, c->ff_coord.p, pc.data(), pc.size() * sizeof(int));
    }
    const cplx gam = gamma_h_of(beta, c->mh);
    const double mh = c->mh.real();
    std::vector<double> kd(static_cast<size_t>(n_energy)), scale(static_cast<size_t>(nrhs));
    for (int e = 0; e < n_energy; ++e) {
        const double k0 = energy_eV[e] / kHbarC, k = mh * k0;
        kd[size_t(e)] = k * c->d;
        const double Pi = 4.0 * kAlphaFs * k0 * k0 / (kPi * kHbarC * std::pow(beta, 4));
        const double sc = Pi / (mh * mh * std::norm(gam)) * k * k * k / (4.0 * kPi);
        for (int t = 0; t < n_traj; ++t) scale[size_t(e) * n_traj + t] = sc;
    }
    // work space: dirs, weights, kd, scale, dP/dOmega, P_CL, amplitudes
    const size_t bd = size_t(n_dir) * 3 * sizeof(double), bw = size_t(n_dir) * sizeof(double);
    const size_t bk = kd.size() * sizeof(double), bs = scale.size() * sizeof(double);
    const size_t bp = size_t(nrhs) * n_dir * sizeof(double), bc = size_t(nrhs) * sizeof(double);
    const size_t ba = size_t(nrhs) * n_dir * 3 * sizeof(z128);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    c->ff_buf.ensure(up(bd) + up(bw) + up(bk) + up(bs) + up(bp) + up(bc) + up(ba));
    char* base = c->ff_buf.as<char>();
    double* ddir = reinterpret_cast<double*>(base);
    double* dw = reinterpret_cast<double*>(base + up(bd));
    double* dkd = reinterpret_cast<double*>(base + up(bd) + up(bw));
    double* dsc = reinterpret_cast<double*>(base + up(bd) + up(bw) + up(bk));
    double* ddp = reinterpret_cast<double*>(base + up(bd) + up(bw) + up(bk) + up(bs));
    double* dpc = reinterpret_cast<double*>(base + up(bd) + up(bw) + up(bk) + up(bs) + up(bp));
    z128* damp = reinterpret_cast<z128*>(base + up(bd) + up(bw) + up(bk) + up(bs) + up(bp) +
                                         up(bc));
    upload(c, ddir, dir_xyz, bd);
    if (weight) upload(c, dw, weight, bw);
    upload(c, dkd, kd.data(), bk);
    upload(c, dsc, scale.data(), bs);
    dda::launch_ff_amp(static_cast<const z128*>(p_dev), c->ff_coord.as<int>(), g.n_occ, g.nx,
                       g.ny, g.nz, ddir, n_dir, dkd, n_energy, n_traj, damp, c->stream);
    dda::launch_ff_power(damp, ddir, weight ? dw : nullptr, n_dir, dsc, nrhs,
                         dp_domega ? ddp : nullptr, p_cl ? dpc : nullptr, c->stream);
    if (dp_domega)
        DDA_HIP_CHECK(hipMemcpyAsync(dp_domega, ddp, bp, hipMemcpyDeviceToHost, c->stream));
    if (p_cl) DDA_HIP_CHECK(hipMemcpyAsync(p_cl, dpc, bc, hipMemcpyDeviceToHost, c->stream));
    wait_stream(c);
    return DDA_OK;
    DDA_API_END
}

// ----------------------------------------------------- total-loss helpers -----
// Closed forms on the host; no device work.

int dda_free_space_loss(double beta, double mh_re, double mh_im, double* dgamma_dz) {
    DDA_API_BEGIN
    if (!dgamma_dz) throw Error(DDA_EINVAL, "dgamma_dz is NULL");
    if (!std::isfinite(beta) || !std::isfinite(mh_re) || !std::isfinite(mh_im) || beta <= 0.0 ||
        beta >= 1.0 || mh_re <= 0.0)
        throw Error(DDA_EINVAL, "need 0 < beta < 1 and a finite host index with Re m_h > 0");
    if (mh_im != 0.0)
        throw Error(DDA_EINVAL,
                    "the free-space loss W_0 is undefined in an absorbing host (section 2.3)");
    // eq. (29) per unit energy through eq. (36): d Gamma_0/dz = alpha_fs (1 - 1/beta_h^2)
    // / (hbar c) above the Cherenkov threshold beta_h = beta m_h > 1, zero below
    const double bh = beta * mh_re;
    *dgamma_dz = bh > 1.0 ? kAlphaFs * (1.0 - 1.0 / (bh * bh)) / kHbarC : 0.0;
    return DDA_OK;
    DDA_API_END
}

int dda_richardson(const double* d_nm, const double* value, int n, double* at_zero,
                   double* ci95) {
    DDA_API_BEGIN
    if (n < 3 || !d_nm || !value || !at_zero) throw Error(DDA_EINVAL, "need n >= 3 points");
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(d_nm[i] > 0.0) || !std::isfinite(d_nm[i]) || !std::isfinite(value[i]))
            throw Error(DDA_EINVAL, "dipole sizes must be > 0 and values finite");
        dmax = std::max(dmax, d_nm[i]);
    }
    // weighted normal equations for a + b t + c t^2, t = d / dmax (scaled for
    // conditioning), weights t^-6 (errors ~ d^3)
    double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, r[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        const double t = d_nm[i] / dmax, w = 1.0 / (t * t * t * t * t * t);
        const double x[3] = {1.0, t, t * t};
        for (int a = 0; a < 3; ++a) {
            r[a] += w * x[a] * value[i];
            for (int b = 0; b < 3; ++b) M[a][b] += w * x[a] * x[b];
        }
    }
    // inverse of the symmetric 3 x 3 matrix by cofactors
    const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
    if (!(std::abs(det) > 0.0) || !std::isfinite(det))
        throw Error(DDA_EINVAL, "the dipole sizes do not determine a quadratic");
    double Mi[3][3];
    Mi[0][0] = c00 / det;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
    Mi[1][0] = c01 / det;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
    Mi[2][0] = c02 / det;
    Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
    double coef[3];
    for (int a = 0; a < 3; ++a) coef[a] = Mi[a][0] * r[0] + Mi[a][1] * r[1] + Mi[a][2] * r[2];
    *at_zero = coef[0];
    if (ci95) {
        if (n == 3) {
            *ci95 = std::numeric_limits<double>::quiet_NaN();
        } else {
            double s2 = 0.0;
            for (int i = 0; i < n; ++i) {
                const double t = d_nm[i] / dmax, w = 1.0 / (t * t * t * t * t * t);
                const double res = value[i] - (coef[0] + coef[1] * t + coef[2] * t * t);
                s2 += w * res * res;
            }
            s2 /= (n - 3);
            *ci95 = 2.0 * std::sqrt(s2 * Mi[0][0]);
        }
    }
    return DDA_OK;
    DDA_API_END
}

int dda_cl_total(const dda_result* res, int n, double mh_im, double* out) {
    DDA_API_BEGIN
    if (n < 0 || (n > 0 && (!res || !out))) throw Error(DDA_EINVAL, "bad arguments");
    if (mh_im != 0.0)
        throw Error(DDA_EINVAL,
                    "P_CL^tot rests on far-field powers that an absorbing host does not "
                    "define (section 2.6)");
    // eq. (41): P_CL^tot is proportional to C_enh - C_ext + C_sca, with the same
    // prefactor as P_EELS (37), P_ext (48) and P_CL (42)
    for (int i = 0; i < n; ++i) out[i] = res[i].p_eels - res[i].p_ext + res[i].p_cl;
    return DDA_OK;
    DDA_API_END
}

int dda_psf_gauss(const double* energy_eV, const double* p, int n, double fwhm_eV,
                  double* out) {
    DDA_API_BEGIN
    if (n < 1 || !energy_eV || !p || !out) throw Error(DDA_EINVAL, "bad arguments");
    if (!(fwhm_eV > 0.0) || !std::isfinite(fwhm_eV)) throw Error(DDA_EINVAL, "fwhm must be > 0");
    if (n == 1) {
        out[0] = p[0];
        return DDA_OK;
    }
    const double de = (energy_eV[n - 1] - energy_eV[0]) / (n - 1);
    if (!(de > 0.0)) throw Error(DDA_EINVAL, "energies must increase");
    for (int i = 0; i < n; ++i)
        if (std::abs(energy_eV[i] - (energy_eV[0] + i * de)) > 1e-9 * std::abs(de) * n)
            throw Error(DDA_EINVAL, "energies must lie on a uniform grid");
    // Gaussian of unit area and the given full width at half maximum, sampled on
    // the grid; the spectrum is taken as zero outside it (no renormalisation at
    // the ends)
    const double sigma = fwhm_eV / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const double norm = de / (sigma * std::sqrt(2.0 * kPi));
    std::vector<double> tmp(size_t(n), 0.0);
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) {
            const double u = (i - j) * de / sigma;
            acc += p[j] * std::exp(-0.5 * u * u);
        }
        tmp[size_t(i)] = norm * acc;
    }
    for (int i = 0; i < n; ++i) out[i] = tmp[size_t(i)];
    return DDA_OK;
    DDA_API_END
}

int dda_setup(const uint8_t* mask, int nx, int ny, int nz, double d_nm, double mh_re,
              double mh_im, const dda_options* opt, void* hip_stream, dda_ctx** out) {
    DDA_API_BEGIN
    g_last_error.clear();
    if (!out) throw Error(DDA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mask) throw Error(DDA_EINVAL, "mask is NULL");
    if (nx < 1 || ny < 1 || nz < 1 || nx > kMaxSide || ny > kMaxSide || nz > kMaxSide)
        throw Error(DDA_EINVAL, "lattice sides must lie in [1, 256]");
    check_finite(d_nm, "d");
    check_finite(mh_re, "Re m_h");
    check_finite(mh_im, "Im m_h");
    if (d_nm <= 0) throw Error(DDA_EINVAL, "d must be positive");
    if (!(mh_re > 0.0) || mh_im < 0.0)
        throw Error(DDA_EINVAL, "host must be passive: Re m_h > 0, Im m_h >= 0");
    auto c = std::make_unique<dda_ctx>();
    if (opt) c->opt = *opt; else dda_default_options(&c->opt);
    if (c->opt.interaction != DDA_INT_POINT && c->opt.interaction != DDA_INT_IGT)
        throw Error(DDA_EINVAL, "unknown interaction");
    if (c->opt.polarizability < 0 || c->opt.polarizability > 2)
        throw Error(DDA_EINVAL, "unknown polarizability");
    if (c->opt.solver != DDA_SOLVER_BICGSTAB && c->opt.solver != DDA_SOLVER_COCG &&
        c->opt.solver != DDA_SOLVER_QMR)
        throw Error(DDA_EINVAL, "unknown solver");
    if (c->opt.precision != DDA_PREC_FP64 && c->opt.precision != DDA_PREC_MIXED)
        throw Error(DDA_EINVAL, "unknown precision");
    if (!(c->opt.tol > 0.0) || !(c->opt.tol < 1.0)) throw Error(DDA_EINVAL, "tol must lie in (0, 1)");
    if (c->opt.maxit < 1) throw Error(DDA_EINVAL, "maxit must be >= 1");
    c->d = d_nm;
    c->mh = cplx(mh_re, mh_im);
    c->stream = static_cast<hipStream_t>(hip_stream);
    dda::Geo& g = c->g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.mx = choose_fft_len(nx);
    g.my = choose_fft_len(ny);
    g.mz = choose_fft_len(nz);
    const int64_t N = int64_t(nx) * ny * nz;
    std::vector<int> hmap(size_t(N), -1);
    for (int64_t i = 0; i < N; ++i) {
        if (mask[i]) {
            hmap[size_t(i)] = int(c->occ_lin.size());
            c->occ_lin.push_back(int(i));
        }
    }
    g.n_occ = int64_t(c->occ_lin.size());
    c->occ_col.assign(size_t(nx) * ny, 0);
    for (int lin : c->occ_lin) c->occ_col[size_t(lin % (nx * ny))] = 1;
    DDA_HIP_CHECK(hipGetDevice(&c->device));
    dda::einc_scratch_init();  // the no-alloc staging area of this device
    c->max_blocks = std::max({1024, dda::pack_blocks_per_slot(g, 8), dda::pack_blocks_per_slot(g, 16),
                              dda::xy_pack_blocks_per_slot(g),
                              dda::yz_pack_blocks_per_slot(g, 8),
                              dda::yz_pack_blocks_per_slot(g, 16)});
    // uploads go through the context's stream (never the legacy stream, which
    // must not touch a stream another thread is capturing)
    c->map.ensure(size_t(N) * sizeof(int));
    upload(c.get(), c->map.p, hmap.data(), size_t(N) * sizeof(int));
    c->occ.ensure(std::max<size_t>(1, c->occ_lin.size()) * sizeof(int));
    upload(c.get(), c->occ.p, c->occ_lin.data(), c->occ_lin.size() * sizeof(int));
    const int Ls[3] = {g.mx, g.my, g.mz};
    for (int a = 0; a < 3; ++a) {
        const int L = Ls[a];
        std::vector<z128> t128(L);
        std::vector<z64> t64(L);
        for (int t = 0; t < L; ++t) {
            const long double ang = -2.0L * 3.141592653589793238462643383279502884L * t / L;
            t128[t] = z128{double(cosl(ang)), double(sinl(ang))};
            t64[t] = z64{float(cosl(ang)), float(sinl(ang))};
        }
        c->tw128[a].ensure(L * sizeof(z128));
        c->tw64[a].ensure(L * sizeof(z64));
        upload(c.get(), c->tw128[a].p, t128.data(), L * sizeof(z128));
        upload(c.get(), c->tw64[a].p, t64.data(), L * sizeof(z64));
    }
    *out = c.release();
    return DDA_OK;
    DDA_API_END
}

int dda_stream_create(void** stream) {
    DDA_API_BEGIN
    if (!stream) throw Error(DDA_EINVAL, "stream is NULL");
    hipStream_t s = nullptr;
    DDA_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    *stream = s;
    return DDA_OK;
    DDA_API_END
}

int dda_stream_destroy(void* stream) {
    DDA_API_BEGIN
    if (stream) DDA_HIP_CHECK(hipStreamDestroy(static_cast<hipStream_t>(stream)));
    return DDA_OK;
    DDA_API_END
}

int dda_set_host(dda_ctx* c, double mh_re, double mh_im) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    check_finite(mh_re, "Re m_h");
    check_finite(mh_im, "Im m_h");
    if (!(mh_re > 0.0) || mh_im < 0.0)
        throw Error(DDA_EINVAL, "host must be passive: Re m_h > 0, Im m_h >= 0");
    c->mh = cplx(mh_re, mh_im);
    return DDA_OK;
    DDA_API_END
}

int dda_n_occ(const dda_ctx* ctx, int64_t* n_occ) {
    if (!ctx || !n_occ) { g_last_error = "NULL argument"; return DDA_EINVAL; }
    *n_occ = ctx->g.n_occ;
    return DDA_OK;
}

int dda_grid_dims(const dda_ctx* ctx, int* mx, int* my, int* mz) {
    if (!ctx || !mx || !my || !mz) { g_last_error = "NULL argument"; return DDA_EINVAL; }
    *mx = ctx->g.mx; *my = ctx->g.my; *mz = ctx->g.mz;
    return DDA_OK;
}

namespace {

// Checks the arguments of an electron-field call; false when there is
// nothing to compute.
bool einc_args(dda_ctx* c, int n_energy, const double* energy_eV, double beta,
               const double* r0_nm, int n_traj, void* einc_dev) {
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (n_energy < 0 || n_traj < 0) throw Error(DDA_EINVAL, "negative batch size");
    if (n_energy == 0 || n_traj == 0 || c->g.n_occ == 0) return false;
    if (!energy_eV || !r0_nm || !einc_dev) throw Error(DDA_EINVAL, "NULL argument");
    check_energies(n_energy, energy_eV);
    check_beta(c, beta);
    host_trajectory_check(c, r0_nm, n_traj);
    return true;
}

// Eq. (25) at every dipole through a device staging area: the energies and
// trajectory points are copied in, the per-energy constants derived on the
// device, then the field kernel runs.  Returns after the stream has passed
// the call, so the caller's host arrays and the staging area are free again.
void einc_staged(dda_ctx* c, int n_energy, const double* energy_eV, double beta,
                 const double* r0_nm, int n_traj, void* einc_dev, const dda::EincStage& st) {
    const cplx gam = gamma_h_of(beta, c->mh);
    const cplx ibg = 1.0 / (beta * gam);
    const cplx ig = cplx(0.0, -1.0) / gam;
    DDA_HIP_CHECK(hipMemcpyAsync(st.energy, energy_eV, size_t(n_energy) * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
    DDA_HIP_CHECK(hipMemcpyAsync(st.r0, r0_nm, size_t(n_traj) * 3 * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
    dda::launch_einc_prep(st.energy, st.sys, n_energy, kHbarC, z128{ibg.real(), ibg.imag()},
                          z128{ig.real(), ig.imag()}, c->stream);
    dda::launch_einc(static_cast<z128*>(einc_dev), c->occ.as<int>(), c->g, c->d, beta, st.sys,
                     st.r0, n_energy, n_traj, c->stream);
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
}

}  // namespace

int dda_einc_electron(dda_ctx* c, int n_energy, const double* energy_eV, double beta,
                      const double* r0_nm, int n_traj, void* einc_dev) {
    DDA_API_BEGIN
    if (!einc_args(c, n_energy, energy_eV, beta, r0_nm, n_traj, einc_dev)) return DDA_OK;
    c->misc.ensure(dda::einc_stage_bytes(size_t(n_energy), size_t(n_traj)));
    einc_staged(c, n_energy, energy_eV, beta, r0_nm, n_traj, einc_dev,
                dda::einc_stage_layout(c->misc.p, size_t(n_energy)));
    return DDA_OK;
    DDA_API_END
}

int dda_einc_electron_noalloc(dda_ctx* c, int n_energy, const double* energy_eV, double beta,
                              const double* r0_nm, int n_traj, void* einc_dev) {
    DDA_API_BEGIN
    if (!einc_args(c, n_energy, energy_eV, beta, r0_nm, n_traj, einc_dev)) return DDA_OK;
    if (n_energy > DDA_EINC_NOALLOC_MAX_ENERGIES || n_traj > DDA_EINC_NOALLOC_MAX_TRAJ)
        throw Error(DDA_EINVAL, "dda_einc_electron_noalloc: at most " +
                                    std::to_string(DDA_EINC_NOALLOC_MAX_ENERGIES) +
                                    " energies and " + std::to_string(DDA_EINC_NOALLOC_MAX_TRAJ) +
                                    " trajectories per call");
    void* base = dda::einc_scratch(c->device);
    if (!base) throw Error(DDA_EDEVICE, "no-alloc staging area not set up on this device");
    einc_staged(c, n_energy, energy_eV, beta, r0_nm, n_traj, einc_dev,
                dda::einc_stage_layout(base, size_t(DDA_EINC_NOALLOC_MAX_ENERGIES)));
    return DDA_OK;
    DDA_API_END
}

static_assert(DDA_EINC_NOALLOC_MAX_ENERGIES == dda::kEincNoallocMaxEnergies &&
                  DDA_EINC_NOALLOC_MAX_TRAJ == dda::kEincNoallocMaxTraj,
              "header and library agree on the no-alloc limits");

int dda_solve(dda_ctx* c, int n_energy, const double* energy_eV, const double* eps_dipole,
              const void* einc_dev, int n_traj, void* p_dev, dda_solve_info* info) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (n_energy < 0 || n_traj < 0) throw Error(DDA_EINVAL, "negative batch size");
    const int64_t nrhs = int64_t(n_energy) * n_traj;
    if (nrhs == 0) return DDA_OK;
    if (c->g.n_occ == 0) {
        if (info)
            for (int64_t i = 0; i < nrhs; ++i) info[i] = dda_solve_info{0, 0, 0.0, DDA_OK};
        return DDA_OK;
    }
    if (!energy_eV || !eps_dipole || !einc_dev || !p_dev) throw Error(DDA_EINVAL, "NULL argument");
    check_energies(n_energy, energy_eV);
    const bool mixed = c->opt.precision == DDA_PREC_MIXED;
    const int64_t nv = c->nv();
    const int spc = systems_per_chunk(c, n_energy, n_traj, mixed);
    int overall = DDA_OK;
    for (int e0 = 0; e0 < n_energy; e0 += spc) {
        const int ns = std::min(spc, n_energy - e0);
        const int nslots = ns * n_traj;
        ensure_slots(c, nslots);
        // slot -> chunk-local system
        {
            std::vector<int> ss(nslots);
            for (int i = 0; i < nslots; ++i) ss[i] = i / n_traj;
            upload(c, c->slot_sys.p, ss.data(), ss.size() * sizeof(int));
        }
        std::vector<DEntry*> ents;
        c->pin_clock = c->use_clock + 1;
        for (int s = 0; s < ns; ++s) ents.push_back(get_D(c, energy_eV[e0 + s], mixed));
        compute_material(c, energy_eV, eps_dipole, e0, ns, true, mixed, nullptr);
        c->G.ensure(size_t(nslots) * dda::grid_elems(c->g) * sizeof(z128));
        const auto* b = static_cast<const z128*>(einc_dev) + int64_t(e0) * n_traj * nv;
        auto* x = static_cast<z128*>(p_dev) + int64_t(e0) * n_traj * nv;
        std::vector<int> iters, mvs, status;
        std::vector<double> relres;
        const size_t q = size_t(nslots) * nv;
        if (c->opt.solver == DDA_SOLVER_COCG || c->opt.solver == DDA_SOLVER_QMR) {
            const bool qmr = c->opt.solver == DDA_SOLVER_QMR;
            const size_t extra = qmr ? 2 : 0;  // QMR keeps two direction vectors more
            auto dptr64 = upload_dptrs<double>(c, ents);
            std::vector<dda_solve_info> inf;
            if (!mixed) {
                c->vec128.ensure((4 + extra) * q * sizeof(z128));
                auto* V = c->vec128.as<z128>();
                CocgBufs<double> B{ctx_work(c), c->act.ptr(), c->slot_sys.as<int>(), b, x, V,
                                   V + q, V + 2 * q, nullptr, V + 3 * q, dptr64,
                                   c->ainv128.as<z128>(), dptr64, c->ainv128.as<z128>()};
                if (qmr) {
                    B.pa = V + 4 * q;
                    B.pb = V + 5 * q;
                    B.qmr = true;
                }
                run_cocg<double>(c, nslots, B, c->opt.tol, c->opt.maxit, inf);
            } else {
                c->vec128.ensure(q * sizeof(z128));
                c->vec64.ensure((4 + extra) * q * sizeof(z64));
                auto* U = c->vec64.as<z64>();
                auto dptr32 = upload_dptrs<float>(c, ents);
                CocgBufs<float> B{ctx_work(c), c->act.ptr(), c->slot_sys.as<int>(), b, x, U,
                                  U + q, U + 2 * q, U + 3 * q, c->vec128.as<z128>(), dptr32,
                                  c->ainv64.as<z64>(), dptr64, c->ainv128.as<z128>()};
                if (qmr) {
                    B.pa = U + 4 * q;
                    B.pb = U + 5 * q;
                    B.qmr = true;
                }
                run_cocg<float>(c, nslots, B, c->opt.tol, c->opt.maxit, inf);
            }
            for (const auto& i : inf) {
                iters.push_back(i.iters);
                mvs.push_back(i.matvecs);
                relres.push_back(i.rel_residual);
                status.push_back(i.status);
            }
        } else if (!mixed) {
            c->vec128.ensure(size_t(6) * q * sizeof(z128));
            auto* V = c->vec128.as<z128>();
            Vecs<double> w{V, V + q, V + 2 * q, V + 3 * q, V + 4 * q, V + 5 * q};
            auto dptr = upload_dptrs<double>(c, ents);
            run_bicgstab<double>(c, nslots, b, x, w, c->opt.tol, c->opt.maxit, true, dptr,
                                 c->ainv128.as<z128>(), iters, mvs, status, relres);
        } else {
            auto dptr64 = upload_dptrs<double>(c, ents);
            auto dptr32 = upload_dptrs<float>(c, ents);
            run_mixed(c, nslots, b, x, dptr64, dptr32, iters, mvs, status, relres);
        }
        for (int i = 0; i < nslots; ++i) {
            if (info) info[int64_t(e0) * n_traj + i] = dda_solve_info{iters[i], mvs[i], relres[i], status[i]};
            if (status[i] != DDA_OK && overall == DDA_OK) overall = status[i];
        }
    }
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (overall != DDA_OK) {
        g_last_error = overall == DDA_ENOCONV ? "iteration limit reached before the tolerance"
                                              : "Krylov breakdown";
    }
    return overall;
    DDA_API_END
}

int dda_eels_cl(dda_ctx* c, int n_energy, const double* energy_eV, double beta,
                const double* eps_dipole, const double* r0_nm, int n_traj, const void* einc_dev,
                const void* p_dev, dda_result* out) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (n_energy < 0 || n_traj < 0) throw Error(DDA_EINVAL, "negative batch size");
    const int64_t nrhs = int64_t(n_energy) * n_traj;
    if (nrhs == 0) return DDA_OK;
    if (!out) throw Error(DDA_EINVAL, "out is NULL");
    if (c->g.n_occ == 0) {
        for (int64_t i = 0; i < nrhs; ++i) out[i] = dda_result{0, 0, 0, 0};
        return DDA_OK;
    }
    if (!energy_eV || !eps_dipole || !r0_nm || !einc_dev || !p_dev)
        throw Error(DDA_EINVAL, "NULL argument");
    check_energies(n_energy, energy_eV);
    check_beta(c, beta);
    const cplx gam = gamma_h_of(beta, c->mh);
    const cplx mh = c->mh;
    const int64_t n = c->g.n_occ, nv = c->nv();
    const int spc = systems_per_chunk(c, n_energy, n_traj, false);
    for (int e0 = 0; e0 < n_energy; e0 += spc) {
        const int ns = std::min(spc, n_energy - e0);
        const int nslots = ns * n_traj;
        ensure_slots(c, nslots);
        {
            std::vector<int> ss(nslots);
            for (int i = 0; i < nslots; ++i) ss[i] = i / n_traj;
            upload(c, c->slot_sys.p, ss.data(), ss.size() * sizeof(int));
        }
        std::vector<DEntry*> ents;
        c->pin_clock = c->use_clock + 1;
        for (int s = 0; s < ns; ++s) ents.push_back(get_D(c, energy_eV[e0 + s], false));
        // absorption weights (device) and omega/v per system
        std::vector<double> kv(ns);
        for (int s = 0; s < ns; ++s) kv[s] = energy_eV[e0 + s] / kHbarC / beta;
        c->G.ensure(size_t(nslots) * dda::grid_elems(c->g) * sizeof(z128));
        c->vec128.ensure(size_t(nslots) * nv * sizeof(z128));
        const size_t wb = size_t(ns) * n * sizeof(double), kb = kv.size() * sizeof(double);
        const size_t rb = size_t(n_traj) * 3 * sizeof(double), ob = size_t(nslots) * 8 * sizeof(double);
        c->misc.ensure(wb + kb + rb + ob + 256);
        char* base = c->misc.as<char>();
        double* dw = reinterpret_cast<double*>(base);
        double* dkv = reinterpret_cast<double*>(base + wb);
        double* dr0 = reinterpret_cast<double*>(base + wb + kb);
        double* dout = reinterpret_cast<double*>(base + wb + kb + rb);
        compute_material(c, energy_eV, eps_dipole, e0, ns, false, false, dw);
        DDA_HIP_CHECK(hipMemcpyAsync(dkv, kv.data(), kb, hipMemcpyHostToDevice, c->stream));
        DDA_HIP_CHECK(hipMemcpyAsync(dr0, r0_nm, rb, hipMemcpyHostToDevice, c->stream));
        const auto* P = static_cast<const z128*>(p_dev) + int64_t(e0) * n_traj * nv;
        auto dptr = upload_dptrs<double>(c, ents);
        auto* Y = c->vec128.as<z128>();
        matvec<double>(c, const_cast<z128*>(P), Y, nullptr, nslots, dptr, c->slot_sys.as<int>(),
                       c->ainv128.as<z128>(), dda::PACK_GX);
        dda::loss_sums(static_cast<const z128*>(einc_dev), static_cast<const z128*>(p_dev), Y, dw,
                       c->occ.as<int>(), c->g, c->d, dkv, dr0, n_traj, int64_t(e0) * n_traj,
                       nslots, dout, red_of(c), c->stream);
        std::vector<double> sums(size_t(nslots) * 8);
        DDA_HIP_CHECK(hipMemcpyAsync(sums.data(), dout, ob, hipMemcpyDeviceToHost, c->stream));
        wait_stream(c);
        for (int i = 0; i < nslots; ++i) {
            const int s = i / n_traj;
            const double E = energy_eV[e0 + s];
            const double k0 = E / kHbarC;
            const double Pi = 4.0 * kAlphaFs * k0 * k0 / (kPi * kHbarC * std::pow(beta, 4));
            const double* q = &sums[size_t(i) * 8];
            const cplx Sa(q[0], q[1]), Se(q[2], q[3]), Spy(q[5], q[6]);
            const double Sw = q[4], Spp = q[7];
            const double g2 = std::norm(gam), mh4 = std::norm(mh * mh);
            dda_result r;
            r.p_eels = -Pi * (Sa / ((mh * gam) * (mh * gam))).imag();
            r.p_ext = Pi * (mh * mh * Se).imag() / (mh4 * g2);
            r.p_abs = Pi / (mh4 * g2) * Sw;
            const double kr = (mh * k0).real();
            r.p_cl = Pi * (mh * mh).real() / (mh4 * g2) * (Spy.imag() + (2.0 / 3.0) * kr * kr * kr * Spp);
            out[int64_t(e0) * n_traj + i] = r;
        }
    }
    return DDA_OK;
    DDA_API_END
}

int dda_matvec(dda_ctx* c, double energy_eV, const double* eps_dipole, int precision,
               int interaction_only, const void* x_dev, void* y_dev, int nrhs) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (nrhs < 0) throw Error(DDA_EINVAL, "nrhs < 0");
    if (nrhs == 0 || c->g.n_occ == 0) return DDA_OK;
    if (!x_dev || !y_dev || (!interaction_only && !eps_dipole)) throw Error(DDA_EINVAL, "NULL argument");
    if (nrhs > 65535) throw Error(DDA_EINVAL, "nrhs > 65535");
    check_energies(1, &energy_eV);
    const bool fp32 = precision == DDA_PREC_MIXED;
    if (precision != DDA_PREC_FP64 && precision != DDA_PREC_MIXED) throw Error(DDA_EINVAL, "bad precision");
    ensure_slots(c, nrhs);
    std::vector<int> ss(nrhs, 0);
    upload(c, c->slot_sys.p, ss.data(), ss.size() * sizeof(int));
    c->pin_clock = c->use_clock + 1;
    std::vector<DEntry*> ents{get_D(c, energy_eV, fp32)};
    if (!interaction_only) {
        compute_material(c, &energy_eV, eps_dipole, 0, 1, true, fp32, nullptr);
    } else {
        c->ainv128.ensure(size_t(c->g.n_occ) * sizeof(z128));
        c->ainv64.ensure(size_t(c->g.n_occ) * sizeof(z64));
    }
    c->G.ensure(size_t(nrhs) * dda::grid_elems(c->g) * sizeof(z128));
    if (!fp32) {
        auto dptr = upload_dptrs<double>(c, ents);
        matvec<double>(c, const_cast<z128*>(static_cast<const z128*>(x_dev)),
                       static_cast<z128*>(y_dev), nullptr, nrhs, dptr, c->slot_sys.as<int>(),
                       c->ainv128.as<z128>(), interaction_only ? dda::PACK_GX : dda::PACK_AX);
    } else {
        auto dptr = upload_dptrs<float>(c, ents);
        matvec<float>(c, const_cast<z64*>(static_cast<const z64*>(x_dev)),
                      static_cast<z64*>(y_dev), nullptr, nrhs, dptr, c->slot_sys.as<int>(),
                      c->ainv64.as<z64>(), interaction_only ? dda::PACK_GX : dda::PACK_AX);
    }
    return DDA_OK;
    DDA_API_END
}

int dda_workspace_bytes(const dda_ctx* c, int n_slots, size_t* bytes) {
    DDA_API_BEGIN
    if (!c || !bytes) throw Error(DDA_EINVAL, "NULL argument");
    if (n_slots < 0) throw Error(DDA_EINVAL, "n_slots < 0");
    // the slots, plus the full-grid FP64 scratch of a D build (one per context)
    *bytes = size_t(n_slots) * engine_slot_bytes(c, c->opt.precision == DDA_PREC_MIXED) +
             (n_slots > 0 ? size_t(dda::dgrid_elems(c->g)) * sizeof(z128) : 0);
    return DDA_OK;
    DDA_API_END
}

int dda_engine_open(dda_ctx* c, int max_slots) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (c->engine) throw Error(DDA_EINVAL, "an engine is already open on this context");
    engine_open(c, max_slots);
    return DDA_OK;
    DDA_API_END
}

int dda_engine_submit_lattice(dda_ctx* c, dda_ctx* lat, int64_t tag, double energy_eV,
                              const double* eps_dipole, const void* einc_dev, void* p_dev) {
    DDA_API_BEGIN
    if (!c || !c->engine) throw Error(DDA_EINVAL, "no engine open on this context");
    if (!lat || !eps_dipole || !einc_dev || !p_dev) throw Error(DDA_EINVAL, "NULL argument");
    if (lat != c) {
        if (lat->g.nx != c->g.nx || lat->g.ny != c->g.ny || lat->g.nz != c->g.nz ||
            lat->d != c->d)
            throw Error(DDA_EINVAL, "the lattice's box or dipole size differs from the engine's");
        if (lat->opt.polarizability != c->opt.polarizability ||
            lat->opt.interaction != c->opt.interaction)
            throw Error(DDA_EINVAL, "the lattice's polarizability or interaction differs");
        if (lat->g.n_occ > c->g.n_occ)
            throw Error(DDA_EINVAL, "the lattice has more dipoles than an engine slot holds");
        if (lat->g.n_occ == 0) throw Error(DDA_EINVAL, "the lattice has no dipoles");
    }
    check_energies(1, &energy_eV);
    const size_t n = size_t(lat->g.n_occ);
    Pending pd{tag, energy_eV, lat->mh, std::vector<double>(eps_dipole, eps_dipole + 2 * n),
               static_cast<const z128*>(einc_dev), static_cast<z128*>(p_dev), lat};
    for (double v : pd.eps)
        if (!std::isfinite(v)) throw Error(DDA_EINVAL, "permittivity is not finite");
    // the engine's stream copies einc at admission: what the lattice's stream
    // queued (the field itself) must have run
    if (lat != c) DDA_HIP_CHECK(hipStreamSynchronize(lat->stream));
    std::lock_guard<std::mutex> lk(c->engine->mu);
    c->engine->queue.push_back(std::move(pd));
    return DDA_OK;
    DDA_API_END
}

int dda_engine_submit(dda_ctx* c, int64_t tag, double energy_eV, const double* eps_dipole,
                      const void* einc_dev, void* p_dev) {
    return dda_engine_submit_lattice(c, c, tag, energy_eV, eps_dipole, einc_dev, p_dev);
}

int dda_engine_poll(dda_ctx* c, int max_intervals, int64_t* tags, dda_solve_info* info,
                    int capacity, int* n_done) {
    DDA_API_BEGIN
    if (!c || !c->engine) throw Error(DDA_EINVAL, "no engine open on this context");
    if (!n_done || (capacity > 0 && (!tags || !info)) || capacity < 0 || max_intervals < 0)
        throw Error(DDA_EINVAL, "bad arguments");
    Engine& E = *c->engine;
    if (E.mixed) engine_poll<float>(c, E, max_intervals);
    else engine_poll<double>(c, E, max_intervals);
    int k = 0;
    while (k < capacity && !E.done.empty()) {
        tags[k] = E.done.front().first;
        info[k] = E.done.front().second;
        E.done.pop_front();
        E.publish();
        ++k;
    }
    *n_done = k;
    return DDA_OK;
    DDA_API_END
}

int dda_engine_status(dda_ctx* c, int* queued, int* running, int* finished) {
    DDA_API_BEGIN
    if (!c || !c->engine || !queued || !running || !finished)
        throw Error(DDA_EINVAL, "bad arguments");
    Engine& E = *c->engine;
    {
        std::lock_guard<std::mutex> lk(E.mu);
        *queued = int(E.queue.size());
    }
    *running = E.n_running.load(std::memory_order_relaxed);
    *finished = E.n_done.load(std::memory_order_relaxed);
    return DDA_OK;
    DDA_API_END
}

int dda_engine_close(dda_ctx* c) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (!c->engine) return DDA_OK;
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
    for (auto& sr : c->engine->slots) engine_release(c, sr);
    c->engine.reset();
    return DDA_OK;
    DDA_API_END
}

int dda_tuning(const dda_ctx* c, int precision, int* zconv_tx, int* mid_tx, int* yz_threads,
               double* t_default_ms, double* t_best_ms) {
    DDA_API_BEGIN
    if (!c || !zconv_tx || !mid_tx || !yz_threads || !t_default_ms || !t_best_ms)
        throw Error(DDA_EINVAL, "NULL argument");
    if (precision != DDA_PREC_FP64 && precision != DDA_PREC_MIXED)
        throw Error(DDA_EINVAL, "bad precision");
    const TuneVal& tv = c->tune[precision == DDA_PREC_FP64 ? 1 : 0];
    *zconv_tx = tv.zconv_tx;
    *mid_tx = tv.mid_tx;
    *yz_threads = tv.yz_threads;
    *t_default_ms = tv.t_default_ms;
    *t_best_ms = tv.t_best_ms;
    return tv.done ? DDA_OK : 1;
    DDA_API_END
}

int dda_set_tuning(dda_ctx* c, int precision, int zconv_tx, int mid_tx, int yz_threads) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    if (precision != DDA_PREC_FP64 && precision != DDA_PREC_MIXED)
        throw Error(DDA_EINVAL, "bad precision");
    const int csize = precision == DDA_PREC_FP64 ? 16 : 8;
    const dda::Geo& g = c->g;
    auto allowed = [](int v, const std::vector<int>& cands) {
        return v == 0 || std::find(cands.begin(), cands.end(), v) != cands.end();
    };
    const bool ok =
        csize == 16
            ? allowed(zconv_tx, dda::zconv_tx_candidates<double>(g.mz)) &&
                  allowed(mid_tx, dda::mid_tx_candidates<double>(g.my))
            : allowed(zconv_tx, dda::zconv_tx_candidates<float>(g.mz)) &&
                  allowed(mid_tx, dda::mid_tx_candidates<float>(g.my));
    if (!ok || !allowed(yz_threads, dda::yz_thread_candidates(g.my)))
        throw Error(DDA_EINVAL, "tile choice not among the candidates for this grid");
    TuneVal& tv = c->tune[csize == 16 ? 1 : 0];
    tv = TuneVal{};
    tv.done = true;
    tv.zconv_tx = zconv_tx;
    tv.mid_tx = mid_tx;
    tv.yz_threads = yz_threads;
    c->graph.drop();
    return DDA_OK;
    DDA_API_END
}

int dda_set_timing(dda_ctx* c, int enabled) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    flush_timer(c);
    c->timing = enabled != 0;
    c->timing_mask = (enabled == 1) ? 0xffu : unsigned(enabled) & 0xffu;
    for (int k = 0; k < kNumKernels; ++k) {
        c->timer.total_ms[k] = 0;
        c->timer.count[k] = 0;
        c->timer.units[k] = 0;
    }
    return DDA_OK;
    DDA_API_END
}

int dda_kernel_time(dda_ctx* c, const char* name, double* avg_ms, int64_t* launches,
                    double* avg_rhs) {
    DDA_API_BEGIN
    if (!c || !name || !avg_ms || !launches || !avg_rhs) throw Error(DDA_EINVAL, "NULL argument");
    flush_timer(c);
    for (int k = 0; k < kNumKernels; ++k) {
        if (std::strcmp(name, kKernelNames[k]) == 0) {
            const int64_t n = c->timer.count[k];
            *launches = n;
            *avg_ms = n ? c->timer.total_ms[k] / double(n) : 0.0;
            *avg_rhs = n ? double(c->timer.units[k]) / double(n) : 0.0;
            return DDA_OK;
        }
    }
    throw Error(DDA_EINVAL, "unknown kernel name");
    DDA_API_END
}

int dda_drop_cache(dda_ctx* c) {
    DDA_API_BEGIN
    if (!c) throw Error(DDA_EINVAL, "ctx is NULL");
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
    // entries an engine slot still solves with stay
    c->dspare.clear();
    for (auto it = c->dcache.begin(); it != c->dcache.end();) {
        if (it->second->refs == 0) it = c->dcache.erase(it);
        else ++it;
    }
    return DDA_OK;
    DDA_API_END
}

int dda_destroy(dda_ctx* c) {
    DDA_API_BEGIN
    if (!c) return DDA_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->sync_ev) (void)hipEventDestroy(c->sync_ev);
    if (c->engine)
        for (auto& sr : c->engine->slots) engine_release(c, sr);
    c->engine.reset();
    delete c;
    return DDA_OK;
    DDA_API_END
}

int dda_debug_besselk01(const double* z, int64_t n, double* k0k1) {
    DDA_API_BEGIN
    if (n < 0 || (n > 0 && (!z || !k0k1))) throw Error(DDA_EINVAL, "bad arguments");
    if (n == 0) return DDA_OK;
    DevBuf dz, d0, d1;
    dz.ensure(size_t(n) * sizeof(z128));
    d0.ensure(size_t(n) * sizeof(z128));
    d1.ensure(size_t(n) * sizeof(z128));
    DDA_HIP_CHECK(hipMemcpy(dz.p, z, size_t(n) * sizeof(z128), hipMemcpyHostToDevice));
    dda::launch_besselk01(dz.as<z128>(), d0.as<z128>(), d1.as<z128>(), n, nullptr);
    std::vector<z128> h0(n), h1(n);
    DDA_HIP_CHECK(hipMemcpy(h0.data(), d0.p, size_t(n) * sizeof(z128), hipMemcpyDeviceToHost));
    DDA_HIP_CHECK(hipMemcpy(h1.data(), d1.p, size_t(n) * sizeof(z128), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) {
        k0k1[4 * i] = h0[i].x;
        k0k1[4 * i + 1] = h0[i].y;
        k0k1[4 * i + 2] = h1[i].x;
        k0k1[4 * i + 3] = h1[i].y;
    }
    return DDA_OK;
    DDA_API_END
}

}  // extern "C"
