// C ABI of the spectrally grouped TV reconstruction library (declared in
// include/sgtv.h): argument validation, the two sliced-ELL copies of the
// system matrix, device buffers of the ADMM state and the per-iteration
// launch sequence.
#include <hip/hip_runtime.h>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "sgtv.h"
#include "sgtv_kernels.h"
#include "sgtv_wsnet.h"

// Device buffer of sgtv_backprojection_noalloc: a file-scope array that the
// code object brings to every GPU the library runs on, held until the process
// ends.  Host code must not pass `scratch` itself to a kernel (in host code it
// names a host-side stand-in); it uses the address hipGetSymbolAddress
// returns for the current device, kept per device by scratch_address().
constexpr int64_t kScratchFloats = int64_t(1) << 23;   // 32 MiB
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

thread_local std::string g_err;

// Device address of `scratch` on each device, looked up once per device with
// that device current (at the first sgtv_create on it).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int device, float **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Spare floats after every vector that the tiled products gather from: the
// kernels stage whole float4 groups, which may run past the last element.
constexpr int64_t kVecPad = 32;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? SGTV_ENOMEM : SGTV_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);                                          \
    } while (0)

// A range of caller-owned device memory handed out in 256-byte aligned
// pieces (bump allocation; `used` is reset when the section is filled anew).
// A counting arena hands out no memory: it only adds up what would be taken.
constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    bool count = false;
};

// While set (ArenaScope), DBuf::alloc takes its memory from this arena
// instead of hipMalloc.
thread_local Arena *t_arena = nullptr;

struct ArenaScope {
    Arena *prev;
    ArenaScope(Arena *a, bool reset) : prev(t_arena) {
        if (a && reset) a->used = 0;
        t_arena = a;
    }
    ~ArenaScope() { t_arena = prev; }
};

bool counting() { return t_arena && t_arena->count; }

// Device allocation: owned (hipMalloc / hipFree) or borrowed from an arena.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), bytes(o.bytes), borrowed(o.borrowed) {
        o.p = nullptr; o.bytes = 0; o.borrowed = false;
    }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; bytes = o.bytes; borrowed = o.borrowed;
            o.p = nullptr; o.bytes = 0; o.borrowed = false;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (p && !borrowed) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        borrowed = false;
    }
    hipError_t alloc(size_t n) {
        release();
        if (Arena *a = t_arena) {
            const size_t off = align_up(a->used), need = n ? n : 16;
            if (!a->count && off + need > a->cap) return hipErrorOutOfMemory;
            a->used = off + need;
            // a counting arena gives a non-null placeholder that is never dereferenced
            p = a->count ? reinterpret_cast<void *>(kAlign) : a->base + off;
            bytes = n;
            borrowed = true;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(&p, n ? n : 16);
        if (e == hipSuccess) bytes = n;
        else p = nullptr;
        return e;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Copy n elements from caller memory (host or device) into a host vector.
template <class T>
hipError_t fetch(std::vector<T> &dst, const T *src, int64_t n, int mem_kind) {
    dst.resize(static_cast<size_t>(n));
    if (n == 0) return hipSuccess;
    if (mem_kind == SGTV_HOST) {
        std::memcpy(dst.data(), src, sizeof(T) * static_cast<size_t>(n));
        return hipSuccess;
    }
    return hipMemcpy(dst.data(), src, sizeof(T) * static_cast<size_t>(n), hipMemcpyDeviceToHost);
}

template <class T>
hipError_t upload(DBuf &dst, const std::vector<T> &src) {
    hipError_t e = dst.alloc(sizeof(T) * src.size());
    if (e != hipSuccess) return e;
    if (src.empty() || counting()) return hipSuccess;
    return hipMemcpy(dst.p, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

// Round-to-nearest-even float -> bfloat16 code (finite inputs).
uint16_t to_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

// Round-to-nearest-even float -> IEEE binary16 code.
uint16_t to_f16(float x) {
    _Float16 h = static_cast<_Float16>(x);
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

// Sliced-ELL packing of n lines given line pointers (CSR-like) into 64-line
// slices, depth padded to a multiple of 4; see sgtv::Sell for the layout.
template <class V>
void pack_sell(int64_t n_lines, const std::vector<int64_t> &lptr, const std::vector<int32_t> &lidx,
               const std::vector<V> &lval, std::vector<int64_t> &sptr, std::vector<int32_t> &idx,
               std::vector<V> &val) {
    const int64_t n_slices = (n_lines + sgtv::kSliceRows - 1) / sgtv::kSliceRows;
    sptr.assign(static_cast<size_t>(n_slices + 1), 0);
    for (int64_t k = 0; k < n_slices; ++k) {
        int64_t width = 0;
        for (int64_t l = k * 64; l < std::min(n_lines, (k + 1) * 64); ++l)
            width = std::max(width, lptr[l + 1] - lptr[l]);
        width = (width + 3) / 4 * 4;
        sptr[k + 1] = sptr[k] + width * 64;
    }
    idx.assign(static_cast<size_t>(sptr[n_slices]), 0);
    val.assign(static_cast<size_t>(sptr[n_slices]), V(0));
    for (int64_t k = 0; k < n_slices; ++k) {
        for (int64_t l = k * 64; l < std::min(n_lines, (k + 1) * 64); ++l) {
            const int64_t lane = l - k * 64;
            for (int64_t t = 0; t < lptr[l + 1] - lptr[l]; ++t) {
                const int64_t pos = sptr[k] + (t / 4) * 256 + lane * 4 + (t % 4);
                idx[pos] = lidx[lptr[l] + t];
                val[pos] = lval[lptr[l] + t];
            }
        }
    }
}

struct Tiled {
    DBuf pk, val, goff, poff, slot;
    sgtv::TileMap map{};
};

// Parameters of one tiled product, after automatic choices.
struct TileParams {
    int rw, waves, cb, ns;
};

int64_t next_pow2(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Automatic schedule: column blocks of up to 16380 entries, slabs so that one
// slab of the gathered vector is at most 2 MiB (an XCD's 4 MiB L2 keeps it
// next to the streamed entries), then more slabs and fewer rows per wave until
// the grid has at least 256 workgroups (one per CU).
TileParams choose_tiles(int64_t n_rows, int64_t n_cols, int waves, int rw, int cb, int ns) {
    TileParams t;
    t.waves = waves > 0 ? waves : 16;
    // 16380 = the widest block of the 24-bit index format (a multiple of 4
    // below 2^14, leaving one code for the zero slot)
    t.cb = cb > 0 ? cb : static_cast<int>(std::min<int64_t>(16380, std::max<int64_t>(4, next_pow2(n_cols))));
    const int64_t ncb = (n_cols + t.cb - 1) / t.cb;
    if (ns > 0) {
        t.ns = ns;
    } else {
        int64_t want = next_pow2((n_cols * 4 + (2 << 20) - 1) >> 21);
        t.ns = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({want, 8, ncb})));
    }
    if (t.ns > ncb) t.ns = static_cast<int>(std::max<int64_t>(1, ncb));
    if (rw > 0) {
        t.rw = rw;
    } else {
        // until there is a tile for every CU: more slabs first (up to 8, each
        // slab keeps its XCDs and its slice of the vector in L2), then shorter
        // tiles (long lists keep the packing dense)
        int r = 1024;
        auto tiles = [&](int rr) { return ((n_rows + int64_t(t.waves) * rr - 1) / (int64_t(t.waves) * rr)) * t.ns; };
        while (tiles(r) < 256) {
            if (ns <= 0 && t.ns < 8 && 2 * t.ns <= ncb) t.ns *= 2;
            else if (r > 64) r >>= 1;
            else break;
        }
        t.rw = r;
    }
    return t;
}

// LDS of a workgroup of the tiled product; idx24: the inner loop reads 24-bit
// indices where the tile fits them
size_t tile_lds_bytes(const TileParams &t, bool idx24) {
    return sgtv::tiled_lds_bytes(t.waves, t.rw, t.cb, idx24 && sgtv::idx24_fits(t.rw, t.cb));
}

// Wall times of the steps of the host-side packing, printed to stderr when
// SGTV_SETUP_TIMES is set (diagnostics).
struct SetupClock {
    bool on = std::getenv("SGTV_SETUP_TIMES") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char *what) {
        if (!on) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[sgtv setup] %-28s %8.3f s\n", what, std::chrono::duration<double>(now - t).count());
        t = now;
    }
};

// Threads of the host-side packing: SGTV_HOST_THREADS when it is set to a
// positive count (at most 64), else up to 16 and no more than the host has.
// The packed arrays do not depend on it.
int64_t host_threads() {
    if (const char *e = std::getenv("SGTV_HOST_THREADS")) {
        const long n = std::strtol(e, nullptr, 10);
        if (n >= 1) return std::min<long>(n, 64);
    }
    return std::max<int64_t>(1, std::min<int64_t>(16, std::thread::hardware_concurrency()));
}

// Calls work(first, step) on up to host_threads() threads, first = 0 .. n - 1
// and step = n, so that each worker takes every nth item of its own loop over
// n_items items; an exception in any worker (an allocation that failed) is
// rethrown as std::bad_alloc once all have finished.  Workers that cannot be
// started run in the caller.
template <class Fn>
void on_threads(int64_t n_items, Fn work) {
    const int64_t nth = std::max<int64_t>(1, std::min<int64_t>(host_threads(), n_items));
    std::atomic<bool> failed{false};
    auto run = [&](int64_t first) {
        try {
            work(first, nth);
        } catch (...) {
            failed = true;
        }
    };
    std::vector<std::thread> pool;
    for (int64_t k = 1; k < nth; ++k) {
        try {
            pool.emplace_back(run, k);
        } catch (...) {
            run(k);
        }
    }
    run(0);
    for (auto &th : pool) th.join();
    if (failed) throw std::bad_alloc();
}

// The columns of a CSR matrix: cp (J + 1 offsets), the rows of every column
// in ascending order (cidx) and the values alongside (cv).  Each worker owns
// a range of columns: it counts them, then, after the prefix sum, passes over
// the rows in order and places the entries of its columns, so every column
// list is written by one worker in row order whatever the thread count.
template <class V>
void transpose_csr(int64_t I, int64_t J, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
                   const std::vector<V> &av, std::vector<int64_t> &cp, std::vector<int32_t> &cidx,
                   std::vector<V> &cv) {
    const int64_t nnz = rp[I];
    const int64_t nw = std::max<int64_t>(1, std::min<int64_t>(host_threads(), J));
    cp.assign(static_cast<size_t>(J + 1), 0);
    cidx.resize(static_cast<size_t>(nnz));
    cv.resize(static_cast<size_t>(nnz));
    on_threads(nw, [&](int64_t me, int64_t step) {
        for (int64_t w = me; w < nw; w += step) {
            const int64_t c0 = J * w / nw, c1 = J * (w + 1) / nw;
            for (int64_t k = 0; k < nnz; ++k)
                if (ci[k] >= c0 && ci[k] < c1) cp[ci[k] + 1]++;
        }
    });
    for (int64_t j = 0; j < J; ++j) cp[j + 1] += cp[j];
    std::vector<int64_t> next(cp.begin(), cp.end() - 1);
    on_threads(nw, [&](int64_t me, int64_t step) {
        for (int64_t w = me; w < nw; w += step) {
            const int64_t c0 = J * w / nw, c1 = J * (w + 1) / nw;
            for (int64_t i = 0; i < I; ++i)
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                    const int64_t c = ci[k];
                    if (c < c0 || c >= c1) continue;
                    const int64_t pos = next[c]++;
                    cidx[pos] = static_cast<int32_t>(i);
                    cv[pos] = av[k];
                }
        }
    });
}

// Host packing of one tiled product from CSR-like lines (rows of M in order,
// column indices ascending within a row).  V is float or a 16-bit code.
template <class V>
int build_tiled(int64_t n_rows, int64_t n_cols, const std::vector<int64_t> &rp,
                const std::vector<int32_t> &ci, const std::vector<V> &vals, const TileParams &t,
                bool idx24, std::vector<int32_t> &pk, std::vector<V> &pv, std::vector<int32_t> &goff,
                std::vector<int32_t> &poff, std::vector<uint16_t> &slot_of, sgtv::TileMap &map) {
    // 24-bit indices: row in 10 bits and column in 14 (up to 1024 rows per
    // wave), or 11 and 13 (up to 2048), with the code cb left for the zero
    // slot.  Their lists are lane-owned: all entries of a row within a list sit
    // in one lane, in row order, so a lane can read every accumulator of a
    // window of entries at once (no other lane touches its rows)
    idx24 = idx24 && sgtv::idx24_fits(t.rw, t.cb);
    const int row_shift = idx24 ? sgtv::idx24_col_bits(t.rw) : 16;
    SetupClock clk;
    const int64_t RB = static_cast<int64_t>(t.waves) * t.rw;
    const int64_t n_rb = (n_rows + RB - 1) / RB;
    const int64_t ncb = (n_cols + t.cb - 1) / t.cb;
    const int ns = t.ns;
    std::vector<int> slab_begin(ns + 1);
    for (int k = 0; k <= ns; ++k) slab_begin[k] = static_cast<int>((k * ncb) / ns);
    int cbs_max = 0;
    for (int k = 0; k < ns; ++k) cbs_max = std::max(cbs_max, slab_begin[k + 1] - slab_begin[k]);
    std::vector<int> slab_of(static_cast<size_t>(ncb));
    for (int k = 0; k < ns; ++k)
        for (int b = slab_begin[k]; b < slab_begin[k + 1]; ++b) slab_of[b] = k;
    const int64_t n_lists = n_rb * ns * cbs_max * t.waves;
    // 24-bit lists: in every tile (row block, slab) the rows of the row block
    // are dealt to the waves so that each wave's share of every column block is
    // as even as possible (every block ends at a barrier, where all waves wait
    // for the longest list).  Greedy: rows by decreasing entry count, each to
    // the wave with room whose loads on the row's blocks are smallest (ties:
    // smaller total, then lower wave).  slot_of[tile * RB + i] is the slot
    // w * rw + l of row offset i (the kernel writes the row sums out in row
    // order through it).  The 32-bit lists, and schedules whose per-row-block
    // counts would pass 2^24 (tiny column blocks of a large matrix), keep row
    // offset i in slot i.
    slot_of.clear();
    const bool balance = idx24 && static_cast<int64_t>(ns) * RB * cbs_max <= (int64_t(1) << 24);
    if (balance) {
        slot_of.assign(static_cast<size_t>(n_rb * ns * RB), 0);
        // row blocks are independent: each worker takes every nth one
        on_threads(n_rb, [&](int64_t first, int64_t step) {
            std::vector<int32_t> cnt(static_cast<size_t>(ns) * RB * cbs_max), tot(static_cast<size_t>(RB));
            std::vector<int32_t> order(static_cast<size_t>(RB)), bucket;
            std::vector<int64_t> load(static_cast<size_t>(t.waves) * cbs_max), wtot(t.waves);
            std::vector<int32_t> filled(t.waves);
            std::vector<int32_t> nzc, nzn;
            for (int64_t rb = first; rb < n_rb; rb += step) {
                std::fill(cnt.begin(), cnt.end(), 0);
                for (int64_t i = 0; i < RB && rb * RB + i < n_rows; ++i)
                    for (int64_t k = rp[rb * RB + i]; k < rp[rb * RB + i + 1]; ++k) {
                        const int64_t cbi = ci[k] / t.cb;
                        const int slab = slab_of[cbi];
                        cnt[(static_cast<size_t>(slab) * RB + i) * cbs_max + (cbi - slab_begin[slab])]++;
                    }
                for (int slab = 0; slab < ns; ++slab) {
                    const int32_t *n = cnt.data() + static_cast<size_t>(slab) * RB * cbs_max;
                    int32_t tmax = 0;
                    for (int64_t i = 0; i < RB; ++i) {
                        int32_t v = 0;
                        for (int c = 0; c < cbs_max; ++c) v += n[i * cbs_max + c];
                        tot[i] = v;
                        tmax = std::max(tmax, v);
                    }
                    // counting sort by decreasing total, stable in row order
                    bucket.assign(static_cast<size_t>(tmax) + 2, 0);
                    for (int64_t i = 0; i < RB; ++i) bucket[tmax - tot[i] + 1]++;
                    for (int32_t v = 1; v <= tmax + 1; ++v) bucket[v] += bucket[v - 1];
                    for (int64_t i = 0; i < RB; ++i) order[bucket[tmax - tot[i]]++] = static_cast<int32_t>(i);
                    std::fill(load.begin(), load.end(), 0);
                    std::fill(wtot.begin(), wtot.end(), 0);
                    std::fill(filled.begin(), filled.end(), 0);
                    const int64_t tile = rb * ns + slab;
                    for (int64_t o = 0; o < RB; ++o) {
                        const int64_t i = order[o];
                        nzc.clear();
                        nzn.clear();
                        for (int c = 0; c < cbs_max; ++c)
                            if (n[i * cbs_max + c]) {
                                nzc.push_back(c);
                                nzn.push_back(n[i * cbs_max + c]);
                            }
                        int best = -1;
                        int64_t best_key = 0;
                        for (int w = 0; w < t.waves; ++w) {
                            if (filled[w] == t.rw) continue;
                            int64_t key = 0;
                            const int64_t *lw = load.data() + static_cast<size_t>(w) * cbs_max;
                            for (size_t u = 0; u < nzc.size(); ++u) key += lw[nzc[u]] * nzn[u];
                            if (best < 0 || key < best_key || (key == best_key && wtot[w] < wtot[best])) {
                                best = w;
                                best_key = key;
                            }
                        }
                        const int64_t slot = static_cast<int64_t>(best) * t.rw + filled[best]++;
                        slot_of[static_cast<size_t>(tile * RB + i)] = static_cast<uint16_t>(slot);
                        int64_t *lw = load.data() + static_cast<size_t>(best) * cbs_max;
                        for (size_t u = 0; u < nzc.size(); ++u) lw[nzc[u]] += nzn[u];
                        wtot[best] += tot[i];
                    }
                }
            }
        });
    }
    clk.mark("  rows dealt to waves");
    // slot (wave * rw + row in the wave) of row r in the tile of column c
    auto slot_in_tile = [&](int64_t r, int32_t c) -> int64_t {
        const int64_t rb = r / RB, i = r - rb * RB;
        if (!balance) return i;
        const int slab = slab_of[c / t.cb];
        return slot_of[static_cast<size_t>((rb * ns + slab) * RB + i)];
    };
    auto list_of = [&](int64_t r, int32_t c) -> int64_t {
        const int64_t rb = r / RB;
        const int64_t w = slot_in_tile(r, c) / t.rw;
        const int64_t cbi = c / t.cb;
        const int slab = slab_of[cbi];
        return ((rb * ns + slab) * cbs_max + (cbi - slab_begin[slab])) * t.waves + w;
    };
    std::vector<int32_t> count(static_cast<size_t>(n_lists), 0), run(static_cast<size_t>(n_lists), 0),
        maxrun(static_cast<size_t>(n_lists), 0);
    std::vector<int64_t> last(static_cast<size_t>(n_lists), -1);
    // the lists of a row block hold only its rows: workers take whole row blocks
    on_threads(n_rb, [&](int64_t first, int64_t step) {
        for (int64_t rb = first; rb < n_rb; rb += step)
            for (int64_t r = rb * RB; r < std::min(n_rows, (rb + 1) * RB); ++r)
                for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
                    const int64_t L = list_of(r, ci[k]);
                    count[L]++;
                    run[L] = last[L] == r ? run[L] + 1 : 1;
                    last[L] = r;
                    maxrun[L] = std::max(maxrun[L], run[L]);
                }
    });
    clk.mark("  list counts");
    // idx24: the entries (indices into ci / vals) of every list, in row order
    std::vector<int64_t> lstart, lent;
    std::vector<int16_t> lrow;   // row within the wave of every listed entry
    if (idx24) {
        lstart.assign(static_cast<size_t>(n_lists + 1), 0);
        for (int64_t L = 0; L < n_lists; ++L) lstart[L + 1] = lstart[L] + count[L];
        lent.resize(static_cast<size_t>(lstart[n_lists]));
        lrow.resize(static_cast<size_t>(lstart[n_lists]));
        std::vector<int64_t> cur(lstart.begin(), lstart.end() - 1);
        on_threads(n_rb, [&](int64_t first, int64_t step) {
            for (int64_t rb = first; rb < n_rb; rb += step)
                for (int64_t r = rb * RB; r < std::min(n_rows, (rb + 1) * RB); ++r)
                    for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
                        const int64_t at = cur[list_of(r, ci[k])]++;
                        lent[at] = k;
                        lrow[at] = static_cast<int16_t>(slot_in_tile(r, ci[k]) % t.rw);
                    }
        });
    }
    clk.mark("  list filling");
    // Lane-owned layout of list L: runs of equal rows, longest first (ties in
    // row order), each to the least-loaded lane (ties: lowest lane); a lane
    // keeps its runs in row order.  Fills lane_load[64] and, in lane order,
    // seq (the entries of lane 0, then lane 1, ...) with lane_begin[65];
    // returns the largest load.  Scratch of one worker:
    struct LaneScratch {
        std::vector<int64_t> run_start, run_len, run_order, seq;
        std::vector<int32_t> run_lane, len_count;
        int32_t lane_load[64];
        int64_t lane_begin[65];
    };
    auto lane_owned = [&](int64_t L, LaneScratch &S) -> int64_t {
        std::vector<int64_t> &run_start = S.run_start, &run_len = S.run_len, &run_order = S.run_order,
                             &seq = S.seq;
        std::vector<int32_t> &run_lane = S.run_lane, &len_count = S.len_count;
        int32_t *lane_load = S.lane_load;
        int64_t *lane_begin = S.lane_begin;
        const int64_t b0 = lstart[L], n = lstart[L + 1] - b0;
        run_start.clear();
        run_len.clear();
        int64_t maxlen = 0;
        for (int64_t i = 0; i < n;) {
            int64_t j = i + 1;
            while (j < n && lrow[b0 + j] == lrow[b0 + i]) ++j;
            run_start.push_back(i);
            run_len.push_back(j - i);
            maxlen = std::max(maxlen, j - i);
            i = j;
        }
        const int64_t nr = static_cast<int64_t>(run_start.size());
        // counting sort of the runs by decreasing length (stable)
        len_count.assign(static_cast<size_t>(maxlen + 2), 0);
        for (int64_t q = 0; q < nr; ++q) len_count[maxlen - run_len[q] + 1]++;
        for (int64_t v = 1; v <= maxlen + 1; ++v) len_count[v] += len_count[v - 1];
        run_order.resize(static_cast<size_t>(nr));
        for (int64_t q = 0; q < nr; ++q) run_order[len_count[maxlen - run_len[q]]++] = q;
        // least-loaded lane by a binary heap on key = load * 64 + lane
        int64_t heap[64];
        for (int l = 0; l < 64; ++l) heap[l] = l;
        run_lane.resize(static_cast<size_t>(nr));
        for (int64_t q : run_order) {
            const int64_t top = heap[0];
            const int lane = static_cast<int>(top & 63);
            run_lane[q] = lane;
            heap[0] = top + run_len[q] * 64;
            for (int h = 0;;) {   // sift down
                int m = h, c1 = 2 * h + 1, c2 = 2 * h + 2;
                if (c1 < 64 && heap[c1] < heap[m]) m = c1;
                if (c2 < 64 && heap[c2] < heap[m]) m = c2;
                if (m == h) break;
                std::swap(heap[h], heap[m]);
                h = m;
            }
        }
        for (int l = 0; l < 64; ++l) lane_load[l] = 0;
        for (int64_t q = 0; q < nr; ++q) lane_load[run_lane[q]] += static_cast<int32_t>(run_len[q]);
        lane_begin[0] = 0;
        int64_t ng = 0;
        for (int l = 0; l < 64; ++l) {
            lane_begin[l + 1] = lane_begin[l] + lane_load[l];
            ng = std::max<int64_t>(ng, lane_load[l]);
        }
        seq.resize(static_cast<size_t>(n));
        int64_t fill[64];
        for (int l = 0; l < 64; ++l) fill[l] = lane_begin[l];
        for (int64_t q = 0; q < nr; ++q)
            for (int64_t u = 0; u < run_len[q]; ++u) seq[fill[run_lane[q]]++] = b0 + run_start[q] + u;
        return ng;
    };
    // lists are packed independently: workers take chunks of 256 lists
    const int64_t n_chunks = (n_lists + 255) / 256;
    auto chunk_lists = [&](int64_t first, int64_t step, auto &&fn) {
        for (int64_t ch = first; ch < n_chunks; ch += step)
            for (int64_t L = ch * 256; L < std::min(n_lists, (ch + 1) * 256); ++L) fn(L);
    };
    std::vector<int32_t> ngr(static_cast<size_t>(n_lists));
    on_threads(n_chunks, [&](int64_t first, int64_t step) {
        LaneScratch S;
        chunk_lists(first, step, [&](int64_t L) {
            const int64_t ng = count[L] == 0 ? 0
                               : idx24     ? lane_owned(L, S)
                                           : std::max<int64_t>((count[L] + 63) / 64, maxrun[L]);
            ngr[L] = static_cast<int32_t>(std::min<int64_t>(ng, int64_t(1) << 30));
        });
    });
    clk.mark("  lane layout (sizes)");
    goff.assign(static_cast<size_t>(n_lists + 1), 0);
    int64_t total = 0;
    for (int64_t L = 0; L < n_lists; ++L) {
        goff[L] = static_cast<int32_t>(total);
        total += ngr[L];
        if (total * 64 >= (int64_t(1) << 31)) return fail(SGTV_ESHAPE, "tiled matrix exceeds 2^31 stored entries");
    }
    goff[n_lists] = static_cast<int32_t>(total);
    // one extra all-padding batch at the end: the kernel streams it in place of
    // a batch past the end of a list
    pk.assign(static_cast<size_t>(total * 64 + 256), t.rw << row_shift);
    pv.assign(static_cast<size_t>(total * 64 + 256), V(0));
    auto slot = [&](int64_t L, int64_t g, int64_t lane) -> int64_t {
        const int64_t ng = ngr[L], nb4 = ng / 4;
        const int64_t base = static_cast<int64_t>(goff[L]) * 64;
        return g < nb4 * 4 ? base + (g / 4) * 256 + lane * 4 + (g % 4)
                           : base + nb4 * 256 + (g - nb4 * 4) * 64 + lane;
    };
    if (!idx24) {
        // round robin over the groups: consecutive entries of a row (one list)
        // fall into consecutive groups, so every group holds distinct rows
        std::fill(count.begin(), count.end(), 0);   // reuse as cursor
        on_threads(n_rb, [&](int64_t first, int64_t step) {
            for (int64_t rb = first; rb < n_rb; rb += step)
                for (int64_t r = rb * RB; r < std::min(n_rows, (rb + 1) * RB); ++r) {
                    const int64_t rl = (r % RB) % t.rw;
                    for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
                        const int32_t c = ci[k];
                        const int64_t L = list_of(r, c);
                        const int64_t kk = count[L]++;
                        const int64_t ng = ngr[L];
                        const int64_t pos = slot(L, kk % ng, kk / ng);
                        pk[pos] = static_cast<int32_t>((rl << row_shift) | (c % t.cb));
                        pv[pos] = vals[k];
                    }
                }
        });
    }
    clk.mark("  array fill");
    poff.clear();
    if (idx24) {
        // lane-owned placement: lane l's i-th entry in group i; a lane shorter
        // than the list repeats its last row with value 0 (its running sum is
        // unchanged), an empty lane takes a row absent from the list; padding
        // reads the zero slot (column code cb)
        on_threads(n_chunks, [&](int64_t first, int64_t step) {
            LaneScratch S;
            std::vector<uint8_t> present(static_cast<size_t>(t.rw));
            const int32_t *lane_load = S.lane_load;
            const int64_t *lane_begin = S.lane_begin;
            const std::vector<int64_t> &seq = S.seq;
            chunk_lists(first, step, [&](int64_t L) {
                if (count[L] == 0) return;
                const int64_t ng = lane_owned(L, S);
                std::fill(present.begin(), present.end(), 0);
                for (int64_t i = lstart[L]; i < lstart[L + 1]; ++i) present[lrow[i]] = 1;
                int free_row = 0;
                for (int l = 0; l < 64; ++l) {
                    int32_t last = -1;
                    for (int64_t i = 0; i < lane_load[l]; ++i) {
                        const int64_t at = seq[lane_begin[l] + i];
                        const int64_t k = lent[at];
                        last = lrow[at];
                        const int64_t pos = slot(L, i, l);
                        pk[pos] = static_cast<int32_t>((last << row_shift) | (ci[k] % t.cb));
                        pv[pos] = vals[k];
                    }
                    if (last < 0) {
                        while (present[free_row]) ++free_row;
                        present[free_row] = 1;
                        last = free_row;
                    }
                    for (int64_t i = lane_load[l]; i < ng; ++i)
                        pk[slot(L, i, l)] = static_cast<int32_t>((last << row_shift) | t.cb);
                }
            });
        });
        // repack: per list, whole batches as three dwords per lane (a plane of
        // 64 dword pairs, then a plane of 64 dwords), then the remaining groups
        // one dword per entry
        poff.assign(static_cast<size_t>(n_lists + 1), 0);
        int64_t words = 0;
        for (int64_t L = 0; L < n_lists; ++L) {
            poff[L] = static_cast<int32_t>(words);
            const int64_t ng = ngr[L], nb4 = ng / 4;
            words += nb4 * 3 * 64 + (ng - nb4 * 4) * 64;   // super-batches take 3 dwords per batch too
        }
        poff[n_lists] = static_cast<int32_t>(words);
        clk.mark("  lane placement");
        std::vector<int32_t> p24(static_cast<size_t>(words));
        on_threads(n_chunks, [&](int64_t first, int64_t step) {
            chunk_lists(first, step, [&](int64_t L) {
                const int64_t ng = ngr[L], nb4 = ng / 4;
                const int64_t base = static_cast<int64_t>(goff[L]) * 64;
                uint32_t *dst = reinterpret_cast<uint32_t *>(p24.data()) + poff[L];
                const int64_t nsb = nb4 / 4;
                for (int64_t b = 0; b < nb4; ++b)
                    for (int64_t lane = 0; lane < 64; ++lane) {
                        const uint32_t *e = reinterpret_cast<const uint32_t *>(pk.data()) + base + b * 256 + lane * 4;
                        const uint32_t w0 = e[0] | (e[1] << 24);
                        const uint32_t w1 = (e[1] >> 8) | (e[2] << 16);
                        const uint32_t w2 = (e[2] >> 16) | (e[3] << 8);
                        if (b < nsb * 4) {
                            // super-batch sb: words 3t .. 3t + 2 of batch t = b % 4, word i in
                            // plane i / 4, slot i % 4 of the lane's 16 bytes
                            uint32_t *sbp = dst + (b / 4) * 768;
                            const int64_t i0 = 3 * (b % 4);
                            const uint32_t w[3] = {w0, w1, w2};
                            for (int64_t k = 0; k < 3; ++k) {
                                const int64_t i = i0 + k;
                                sbp[(i / 4) * 256 + lane * 4 + (i % 4)] = w[k];
                            }
                        } else {
                            uint32_t *bp = dst + nsb * 768 + (b - nsb * 4) * 192;
                            bp[lane * 2] = w0;
                            bp[lane * 2 + 1] = w1;
                            bp[128 + lane] = w2;
                        }
                    }
                for (int64_t g = nb4 * 4; g < ng; ++g)
                    for (int64_t lane = 0; lane < 64; ++lane)
                        dst[nb4 * 192 + (g - nb4 * 4) * 64 + lane] =
                            static_cast<uint32_t>(pk[base + nb4 * 256 + (g - nb4 * 4) * 64 + lane]);
            });
        });
        // keep the all-padding batch of the 32-bit layout after the repacked
        // lists (the simple loop that reads 24-bit indices never streams it)
        p24.insert(p24.end(), pk.end() - 256, pk.end());
        pk.swap(p24);
        clk.mark("  24-bit repacking");
    }
    map = sgtv::TileMap{};
    map.idx24 = idx24 ? 1 : 0;
    map.n_rows = n_rows;
    map.n_cols = n_cols;
    map.n_rb = n_rb;
    map.pad = idx24 ? static_cast<int64_t>(pk.size()) - 256 : total * 64;
    map.rw = t.rw;
    map.waves = t.waves;
    map.cb = t.cb;
    map.ns = ns;
    map.cbs_max = cbs_max;
    map.variant = 0;
    map.cbits = idx24 ? row_shift : 0;
    for (int k = 0; k <= ns; ++k) map.slab_begin[k] = slab_begin[k];
    return SGTV_OK;
}

// Host image of one tiled copy (what the device buffers will hold).
struct PackedTiled {
    std::vector<int32_t> pk, goff, poff;
    std::vector<float> v32;          // FP32 values ...
    std::vector<uint16_t> v16;       // ... or 16-bit codes
    std::vector<uint16_t> slot;
    sgtv::TileMap map{};
};

template <class V>
int pack_tiled(PackedTiled &T, int64_t n_rows, int64_t n_cols, const std::vector<int64_t> &rp,
               const std::vector<int32_t> &ci, const std::vector<V> &vals, const TileParams &t, bool idx24) {
    std::vector<V> pv;
    if (int e = build_tiled(n_rows, n_cols, rp, ci, vals, t, idx24, T.pk, pv, T.goff, T.poff, T.slot, T.map))
        return e;
    if constexpr (sizeof(V) == 4) T.v32.swap(pv);
    else T.v16.swap(pv);
    return SGTV_OK;
}

// Points a tile map at its device arrays (absent arrays: null).
void point_tiled(Tiled &T) {
    T.map.pk = T.pk.as<int32_t>();
    T.map.val = T.val.p;
    T.map.goff = T.goff.as<int32_t>();
    T.map.poff = T.poff.as<int32_t>();
    T.map.slot = T.slot.as<uint16_t>();
}

int upload_tiled(Tiled &T, const PackedTiled &P) {
    T.map = P.map;
    HIP_TRY(upload(T.pk, P.pk));
    if (!P.v32.empty() || P.v16.empty()) HIP_TRY(upload(T.val, P.v32));
    else HIP_TRY(upload(T.val, P.v16));
    HIP_TRY(upload(T.goff, P.goff));
    if (!P.poff.empty()) HIP_TRY(upload(T.poff, P.poff));
    if (!P.slot.empty()) HIP_TRY(upload(T.slot, P.slot));
    point_tiled(T);
    return SGTV_OK;
}

struct System {
    int64_t I = 0, J = 0, S = 0, nnz = 0;
    int ny = 0, nx = 0, Q = 0, vt = SGTV_F32;
    int format = SGTV_FORMAT_TILED;
    sgtv_schedule sched{};       // resolved schedule
    sgtv::Grid grid{};
    float w4[4] = {1, 1, 1, 1};
    bool wfull = false;
    DBuf rs_ptr, rs_idx, rs_val, cs_ptr, cs_idx, cs_val, colscale, sens, H, wbuf;
    DBuf htab;                   // H0 by neighbour pattern (weights constant per direction)
    int fused_tw = 0, fused_th = 0;   // tile of the fused image and split update (0: not fused)
    int fused_threads = sgtv::kFusedThreads;
    std::vector<int64_t> perm;   // internal row -> caller row (identity for tiles)
    int64_t n_rslices = 0, n_cslices = 0;
    Tiled fwd, back;             // tiled format: A (rows = measurements), A^T (rows = voxels)
    DBuf fpart, bpart;           // per-slab partial sums
    DBuf fcount, bcount;         // arrival counters of the row-block epilogues (zero between launches)

    sgtv::Sell rows() const {
        return {rs_ptr.as<int64_t>(), rs_idx.as<int32_t>(), rs_val.p, nullptr, I, n_rslices};
    }
    sgtv::Sell cols() const {
        return {cs_ptr.as<int64_t>(), cs_idx.as<int32_t>(), cs_val.p,
                vt == SGTV_F32 ? nullptr : colscale.as<float>(), J, n_cslices};
    }
    sgtv::Weights weights() const {
        sgtv::Weights w;
        for (int p = 0; p < 4; ++p) w.w[p] = w4[p];
        w.full = wfull ? wbuf.as<float>() : nullptr;
        return w;
    }
};

// A system packed on the host, not yet on the device: the metadata in S (no
// device buffers) and the host arrays of every buffer.
struct Packed {
    std::unique_ptr<System> S;
    std::vector<float> colscale, H, htab, wf;
    PackedTiled fwd, back;
    size_t fpart_floats = 0, bpart_floats = 0;
    std::vector<int64_t> rsp, csp;
    std::vector<int32_t> rsi, csi;
    std::vector<float> rsv32, csv32;
    std::vector<uint16_t> rsv16, csv16;
};

// Caller-owned device memory of a context, cut into sections that are filled
// independently: the system (matrix copies, H, partial sums, reductions),
// the data (y, r, ratio), the iteration state and the temporaries of single
// calls.
struct Workspace {
    char *base = nullptr;
    size_t size = 0;
    Arena sys, data, state, temp;
};

}  // namespace

struct sgtv_ctx_s;
typedef sgtv_ctx_s Context;

struct sgtv_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    sgtv_schedule want{};        // requested schedule for the next system
    std::unique_ptr<System> sys;
    // data
    bool has_data = false;
    DBuf y, r, ratio;
    double beta = 0.0, rho = 1.0;
    int sweeps = 1;
    int grouping = SGTV_GROUP_SPECTRAL;
    // state: image (double buffered), split state (v, a) double buffered
    DBuf f[2], v[2], a[2], fs;
    int fcur = 0, vcur = 0;
    int64_t k = 0;
    // reductions
    DBuf part, red;
    int64_t part_cap = 0;
    // caller-owned device memory (base null: the library allocates) and a
    // system packed by sgtv_plan_system, waiting for sgtv_commit_system
    Workspace ws;
    std::unique_ptr<Packed> pending;
    int64_t pending_bytes = 0;
    size_t pending_sections[4] = {0, 0, 0, 0};
    // image and split updates in one pass (off by default: slower here, see
    // sgtv_set_fused_update)
    bool fused = false;
    bool epilogues = false;      // tiled products finish their row blocks (ratio, image update)
    // graph replay of iterate(n)
    bool use_graphs = true;
    hipStream_t cap = nullptr;   // capture stream (own, created on first use)
    struct Graph { int n, fcur, vcur, fcur_after, vcur_after; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
    // optional kernel timing: (class, start, end) per launch
    bool profiling = false;
    struct Timed { int cls; hipEvent_t beg, end; };
    std::vector<Timed> timed;
};

namespace {

void drop_graphs(sgtv_ctx_s *c) {
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

int64_t n_groups(const sgtv_ctx_s *c) {
    return c->grouping == SGTV_GROUP_SPECTRAL ? c->sys->S : c->sys->J;
}

bool finite_nonneg(float x) { return std::isfinite(x) && x >= 0.0f; }

// Allocate state buffers sized for the current system and grouping.
int alloc_state(sgtv_ctx_s *c) {
    const System &S = *c->sys;
    const int64_t ng = n_groups(c);
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(c->f[b].alloc(sizeof(float) * (S.J + kVecPad)));
        HIP_TRY(c->v[b].alloc(sizeof(float) * S.J * 4));
        HIP_TRY(c->a[b].alloc(sizeof(float) * ng));
    }
    HIP_TRY(c->fs.alloc(sizeof(float) * (S.J + kVecPad)));
    return SGTV_OK;
}

// Scaled copy sigma .* f used as the gathered vector of the 16-bit forward projection.
int refresh_scaled(sgtv_ctx_s *c) {
    const System &S = *c->sys;
    if (S.vt != SGTV_F32)
        HIP_TRY(sgtv::launch_scale(c->f[c->fcur].as<float>(), S.colscale.as<float>(),
                                   c->fs.as<float>(), S.J, c->stream));
    return SGTV_OK;
}

// d = c = 0 (v = 0, a = 0 in both buffers), k = 0.
int clear_split(sgtv_ctx_s *c) {
    const System &S = *c->sys;
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipMemsetAsync(c->v[b].p, 0, sizeof(float) * S.J * 4, c->stream));
        HIP_TRY(hipMemsetAsync(c->a[b].p, 0, sizeof(float) * n_groups(c), c->stream));
    }
    c->vcur = 0;
    c->k = 0;
    return SGTV_OK;
}

// f = kappa * 1 with kappa = sum(y) / sum(sens), reduced in FP64 on the device.
int uniform_start(sgtv_ctx_s *c) {
    const System &S = *c->sys;
    int64_t nb = 0;
    double *red = c->red.as<double>();
    HIP_TRY(sgtv::launch_sum_f32(c->y.as<float>(), S.I, c->part.as<double>(), c->stream, &nb));
    HIP_TRY(sgtv::launch_reduce(c->part.as<double>(), nb, 1, red + 4, c->stream));
    HIP_TRY(sgtv::launch_sum_f32(S.sens.as<float>(), S.J, c->part.as<double>(), c->stream, &nb));
    HIP_TRY(sgtv::launch_reduce(c->part.as<double>(), nb, 1, red + 5, c->stream));
    c->fcur = 0;
    HIP_TRY(sgtv::launch_fill_ratio(red + 4, red + 5, c->f[0].as<float>(), S.J, c->stream));
    return SGTV_OK;
}

int check_ready(sgtv_ctx_s *c) {
    if (!c) return fail(SGTV_EINVAL, "null context");
    if (!c->sys) return fail(SGTV_ESTATE, "no system set (call sgtv_set_system first)");
    if (!c->has_data) return fail(SGTV_ESTATE, "no data set (call sgtv_set_data first)");
    return SGTV_OK;
}

int check_mem_kind(int mk) {
    if (mk != SGTV_HOST && mk != SGTV_DEVICE) return fail(SGTV_EINVAL, "mem_kind must be SGTV_HOST or SGTV_DEVICE");
    return SGTV_OK;
}

hipMemcpyKind to_caller(int mk) { return mk == SGTV_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice; }
hipMemcpyKind from_caller(int mk) { return mk == SGTV_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice; }

// Upload a validated float array of n values from caller memory into dst.
int stage_floats(DBuf &dst, const float *src, int64_t n, int mk, hipStream_t st,
                 bool (*ok)(float), const char *what) {
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<float> h;
    HIP_TRY(fetch(h, src, n, mk));
    for (int64_t i = 0; i < n; ++i)
        if (!ok(h[i])) return fail(SGTV_EINVAL, std::string(what) + " has an invalid value at index " + std::to_string(i));
    HIP_TRY(dst.alloc(sizeof(float) * n));
    HIP_TRY(hipMemcpyAsync(dst.p, h.data(), sizeof(float) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SGTV_OK;
}

// e = A^T t with the stored values (scaled back for 16-bit codes).
int back_project(const System &S, const float *t, float *e, hipStream_t st) {
    if (S.format == SGTV_FORMAT_TILED) {
        HIP_TRY(sgtv::launch_tiled(S.back.map, S.vt, t, S.bpart.as<float>(), st));
        HIP_TRY(sgtv::launch_back_combine(S.bpart.as<float>(), S.back.map.ns, S.J,
                                          S.vt == SGTV_F32 ? nullptr : S.colscale.as<float>(), e, st));
    } else {
        HIP_TRY(sgtv::launch_back(S.cols(), S.vt, t, e, st));
    }
    return SGTV_OK;
}

// Tile of the fused image and split update: the largest of a few shapes that
// still gives a tile for each of the 256 CUs, else the smallest (small grids
// are latency-bound); its LDS (the tile and its ring, all spectral bins) must
// fit.  SGTV_FUSED_TILE="tw,th" overrides the choice (measurement); tw = 0
// turns the fused pass off.
void choose_fused_tile(int ny, int nx, int Q, int *tw, int *th) {
    *tw = *th = 0;
    if (const char *e = std::getenv("SGTV_FUSED_TILE")) {
        int a = 0, b = 0;
        if (std::sscanf(e, "%d,%d", &a, &b) == 2 && a >= 0 && b >= 0) {
            if (a > 0 && b > 0 && sgtv::fused_lds_bytes(a, b, Q) <= static_cast<size_t>(sgtv::kFusedMaxLds)) {
                *tw = a;
                *th = b;
            }
            return;
        }
    }
    static const int cand[][2] = {{8, 8}, {16, 4}, {8, 4}, {4, 4}, {4, 2}, {2, 2}, {2, 1}, {1, 1}};
    int best_w = 0, best_h = 0;
    for (const auto &c : cand) {
        if (sgtv::fused_lds_bytes(c[0], c[1], Q) > static_cast<size_t>(sgtv::kFusedMaxLds)) continue;
        best_w = c[0];
        best_h = c[1];
        const int64_t tiles = static_cast<int64_t>((nx + c[0] - 1) / c[0]) * ((ny + c[1] - 1) / c[1]);
        if (tiles >= 256) break;
    }
    *tw = best_w;
    *th = best_h;
}

// Validate the system and pack it on the host (no device memory touched).
int pack_system(sgtv_ctx_s *c, Packed &PK, int64_t I, int32_t ny, int32_t nx, int32_t Q,
                const int64_t *row_ptr, const int32_t *col_idx, const float *val, int64_t nnz, int vt,
                const float *w, int64_t w_len, int mk) {
    PK.S = std::make_unique<System>();
    System *S = PK.S.get();
    SetupClock clk;
    S->I = I; S->ny = ny; S->nx = nx; S->Q = Q; S->vt = vt; S->nnz = nnz;
    S->S = static_cast<int64_t>(ny) * nx;
    S->J = S->S * Q;
    S->grid = sgtv::Grid{ny, nx, Q, S->S, S->J};
    const int64_t J = S->J;

    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<float> av;
    HIP_TRY(fetch(rp, row_ptr, I + 1, mk));
    HIP_TRY(fetch(ci, col_idx, nnz, mk));
    HIP_TRY(fetch(av, val, nnz, mk));
    clk.mark("fetch");
    if (rp[0] != 0 || rp[I] != nnz) return fail(SGTV_ESHAPE, "row_ptr[0] must be 0 and row_ptr[I] must equal nnz");
    for (int64_t i = 0; i < I; ++i)
        if (rp[i + 1] < rp[i]) return fail(SGTV_ESHAPE, "row_ptr decreases at row " + std::to_string(i));
    for (int64_t k = 0; k < nnz; ++k) {
        if (ci[k] < 0 || ci[k] >= J) return fail(SGTV_ESHAPE, "column index out of range at entry " + std::to_string(k));
        if (!finite_nonneg(av[k])) return fail(SGTV_EINVAL, "matrix value not finite and nonnegative at entry " + std::to_string(k));
    }
    // weights
    std::vector<float> wf;
    if (w) {
        HIP_TRY(fetch(wf, w, w_len, mk));
        for (int64_t k = 0; k < w_len; ++k)
            if (!(std::isfinite(wf[k]) && wf[k] > 0.0f)) return fail(SGTV_EINVAL, "weights must be finite and positive");
        if (w_len == 4) {
            for (int p = 0; p < 4; ++p) S->w4[p] = wf[p];
        } else {
            S->wfull = true;
        }
    }
    clk.mark("validation");
    // De Pierro curvature without the penalty factor: H0 = |D|^T |D| 1 (the
    // kernels use rho * H0)
    std::vector<double> Hd(static_cast<size_t>(J), 0.0);
    for (int64_t s = 0; s < S->S; ++s) {
        const int iy = static_cast<int>(s / nx), ix = static_cast<int>(s % nx);
        for (int p = 0; p < 4; ++p) {
            int64_t nb = -1;
            if (p == 0 && ix + 1 < nx) nb = s + 1;
            if (p == 1 && ix > 0) nb = s - 1;
            if (p == 2 && iy + 1 < ny) nb = s + nx;
            if (p == 3 && iy > 0) nb = s - nx;
            for (int q = 0; q < Q; ++q) {
                const double wt = S->wfull ? wf[(s * 4 + p) * Q + q] : S->w4[p];
                const double l1 = nb >= 0 ? 2.0 * wt : wt;
                Hd[s * Q + q] += wt * l1;
                if (nb >= 0) Hd[nb * Q + q] += wt * l1;
            }
        }
    }
    std::vector<float> Hf(Hd.begin(), Hd.end());
    // with weights constant per direction, H0 of a voxel depends only on which
    // of its four neighbours lie in the grid: a table of the 16 patterns
    std::vector<float> htab(16, 0.0f);
    if (!S->wfull) {
        std::vector<char> seen(16, 0);
        for (int64_t s = 0; s < S->S; ++s) {
            const int iy = static_cast<int>(s / nx), ix = static_cast<int>(s % nx);
            const int m = (ix + 1 < nx ? 1 : 0) | (ix > 0 ? 2 : 0) | (iy + 1 < ny ? 4 : 0) | (iy > 0 ? 8 : 0);
            for (int q = 0; q < Q; ++q) {
                const float h = Hf[s * Q + q];
                if (!seen[m]) {
                    htab[m] = h;
                    seen[m] = 1;
                } else if (std::memcmp(&h, &htab[m], sizeof(float)) != 0) {
                    return fail(SGTV_EDEVICE, "curvature differs within one neighbour pattern");
                }
            }
        }
    }

    clk.mark("curvature");
    // column scales and 16-bit codes
    std::vector<float> sigma;
    std::vector<uint16_t> codes;
    if (vt != SGTV_F32) {
        sigma.assign(static_cast<size_t>(J), 0.0f);
        for (int64_t k = 0; k < nnz; ++k) sigma[ci[k]] = std::max(sigma[ci[k]], av[k]);
        codes.resize(static_cast<size_t>(nnz));
        for (int64_t k = 0; k < nnz; ++k) {
            const float sj = sigma[ci[k]];
            const float t = sj > 0.0f ? av[k] / sj : 0.0f;
            codes[k] = vt == SGTV_BF16 ? to_bf16(t) : to_f16(t);
        }
        for (int64_t j = 0; j < J; ++j)
            if (sigma[j] == 0.0f) sigma[j] = 1.0f;   // empty / all-zero column: any scale
        PK.colscale = std::move(sigma);
    }

    S->format = c->want.format;
    S->sched = c->want;
    if (S->format == SGTV_FORMAT_TILED) {
        const sgtv_schedule &q = c->want;
        const TileParams tf = choose_tiles(I, J, q.waves, q.fwd_rows_per_wave, q.fwd_block_cols, q.fwd_slabs);
        const TileParams tb = choose_tiles(J, I, q.waves, q.back_rows_per_wave, q.back_block_cols, q.back_slabs);
        const bool var1 = q.variant <= 1;   // the simple loop, the only one on 24-bit indices
        if (tile_lds_bytes(tf, var1) > 163840 || tile_lds_bytes(tb, var1) > 163840)
            return fail(SGTV_EINVAL, "schedule needs more than 160 KiB of LDS per workgroup");
        S->sched.waves = tf.waves;
        S->sched.fwd_rows_per_wave = tf.rw; S->sched.fwd_block_cols = tf.cb; S->sched.fwd_slabs = tf.ns;
        S->sched.back_rows_per_wave = tb.rw; S->sched.back_block_cols = tb.cb; S->sched.back_slabs = tb.ns;
        S->sched.variant = q.variant > 0 ? q.variant : 1;
        S->perm.resize(static_cast<size_t>(I));
        for (int64_t i = 0; i < I; ++i) S->perm[i] = i;
        // the simple loop (variant 1) reads 24-bit indices where the tile fits them
        const bool i24 = S->sched.variant == 1;
        // transpose (rows ascending within a column) with the values alongside
        std::vector<int64_t> cp;
        std::vector<int32_t> cidx;
        if (vt == SGTV_F32) {
            std::vector<float> cv;
            transpose_csr(I, J, rp, ci, av, cp, cidx, cv);
            clk.mark("transpose");
            if (int e = pack_tiled(PK.fwd, I, J, rp, ci, av, tf, i24)) return e;
            clk.mark("forward copy");
            if (int e = pack_tiled(PK.back, J, I, cp, cidx, cv, tb, i24)) return e;
            clk.mark("back copy");
        } else {
            std::vector<uint16_t> cv;
            transpose_csr(I, J, rp, ci, codes, cp, cidx, cv);
            clk.mark("transpose");
            if (int e = pack_tiled(PK.fwd, I, J, rp, ci, codes, tf, i24)) return e;
            clk.mark("forward copy");
            if (int e = pack_tiled(PK.back, J, I, cp, cidx, cv, tb, i24)) return e;
            clk.mark("back copy");
        }
        PK.fwd.map.variant = S->sched.variant - 1;
        PK.back.map.variant = S->sched.variant - 1;
        S->fwd.map = PK.fwd.map;
        S->back.map = PK.back.map;
        PK.fpart_floats = static_cast<size_t>(I) * tf.ns;
        PK.bpart_floats = static_cast<size_t>(J) * tb.ns;
    } else {
        // internal row order: rows sorted by decreasing length (stable), so that
        // the 64 rows of a slice have nearly equal lengths
        int64_t maxlen = 0;
        for (int64_t i = 0; i < I; ++i) maxlen = std::max(maxlen, rp[i + 1] - rp[i]);
        std::vector<int64_t> cnt(static_cast<size_t>(maxlen + 2), 0);
        for (int64_t i = 0; i < I; ++i) cnt[maxlen - (rp[i + 1] - rp[i])]++;
        std::vector<int64_t> start(static_cast<size_t>(maxlen + 2), 0);
        for (int64_t b = 1; b <= maxlen + 1; ++b) start[b] = start[b - 1] + cnt[b - 1];
        S->perm.assign(static_cast<size_t>(I), 0);
        for (int64_t i = 0; i < I; ++i) S->perm[start[maxlen - (rp[i + 1] - rp[i])]++] = i;

        std::vector<int64_t> lp(static_cast<size_t>(I + 1), 0);
        for (int64_t i = 0; i < I; ++i) {
            const int64_t o = S->perm[i];
            lp[i + 1] = lp[i] + (rp[o + 1] - rp[o]);
        }
        std::vector<int32_t> lidx(static_cast<size_t>(nnz));
        std::vector<int64_t> lsrc(static_cast<size_t>(nnz));   // position in caller CSR
        for (int64_t i = 0; i < I; ++i) {
            const int64_t o = S->perm[i];
            for (int64_t t = 0; t < rp[o + 1] - rp[o]; ++t) {
                lidx[lp[i] + t] = ci[rp[o] + t];
                lsrc[lp[i] + t] = rp[o] + t;
            }
        }
        // columns: counting sort of the internal-order rows, rows ascending within a column
        std::vector<int64_t> cp(static_cast<size_t>(J + 1), 0);
        for (int64_t k = 0; k < nnz; ++k) cp[ci[k] + 1]++;
        for (int64_t j = 0; j < J; ++j) cp[j + 1] += cp[j];
        std::vector<int64_t> cur(cp.begin(), cp.end() - 1);
        std::vector<int32_t> cidx(static_cast<size_t>(nnz));
        std::vector<int64_t> csrc(static_cast<size_t>(nnz));
        for (int64_t i = 0; i < I; ++i)
            for (int64_t k = lp[i]; k < lp[i + 1]; ++k) {
                const int64_t pos = cur[lidx[k]]++;
                cidx[pos] = static_cast<int32_t>(i);
                csrc[pos] = lsrc[k];
            }

        std::vector<int64_t> rsp, csp;
        std::vector<int32_t> rsi, csi;
        if (vt == SGTV_F32) {
            std::vector<float> lv(static_cast<size_t>(nnz)), cv(static_cast<size_t>(nnz));
            for (int64_t k = 0; k < nnz; ++k) { lv[k] = av[lsrc[k]]; cv[k] = av[csrc[k]]; }
            pack_sell(I, lp, lidx, lv, rsp, rsi, PK.rsv32);
            pack_sell(J, cp, cidx, cv, csp, csi, PK.csv32);
        } else {
            std::vector<uint16_t> lv(static_cast<size_t>(nnz)), cv(static_cast<size_t>(nnz));
            for (int64_t k = 0; k < nnz; ++k) { lv[k] = codes[lsrc[k]]; cv[k] = codes[csrc[k]]; }
            pack_sell(I, lp, lidx, lv, rsp, rsi, PK.rsv16);
            pack_sell(J, cp, cidx, cv, csp, csi, PK.csv16);
        }
        if (rsp.back() >= (int64_t(1) << 31) || csp.back() >= (int64_t(1) << 31))
            return fail(SGTV_ESHAPE, "padded matrix exceeds 2^31 entries");
        S->n_rslices = static_cast<int64_t>(rsp.size()) - 1;
        S->n_cslices = static_cast<int64_t>(csp.size()) - 1;
        PK.rsp.swap(rsp);
        PK.rsi.swap(rsi);
        PK.csp.swap(csp);
        PK.csi.swap(csi);
    }
    PK.H.swap(Hf);
    PK.htab.swap(htab);
    if (S->wfull) PK.wf.swap(wf);
    choose_fused_tile(ny, nx, Q, &S->fused_tw, &S->fused_th);
    if (const char *e = std::getenv("SGTV_FUSED_THREADS")) {
        const int t = std::atoi(e);
        if (t == 256 || t == 512 || t == 1024) S->fused_threads = t;
    }
    return SGTV_OK;
}

int compute_sensitivity(sgtv_ctx_s *c, System &S, Arena *temp);

// Arrival counters of the tiled products' row-block epilogues, one per row
// block, cleared here (set-up, never inside a captured graph); every launch
// leaves them at zero again.
int alloc_counters(sgtv_ctx_s *c, System &S) {
    HIP_TRY(S.fcount.alloc(sizeof(uint32_t) * static_cast<size_t>(std::max<int64_t>(S.fwd.map.n_rb, 1))));
    HIP_TRY(S.bcount.alloc(sizeof(uint32_t) * static_cast<size_t>(std::max<int64_t>(S.back.map.n_rb, 1))));
    if (counting()) return SGTV_OK;
    HIP_TRY(hipMemsetAsync(S.fcount.p, 0, S.fcount.bytes, c->stream));
    HIP_TRY(hipMemsetAsync(S.bcount.p, 0, S.bcount.bytes, c->stream));
    return SGTV_OK;
}

// Put a packed system on the device: every buffer is allocated (from the
// current arena, if any; a counting arena only adds up the bytes) and
// filled, and the sensitivity s = A^T 1 is computed with the stored values
// (its vector of ones is a temporary from `temp`, or library memory when
// temp is null).  Leaves the host arrays in PK.
int upload_system(sgtv_ctx_s *c, Packed &PK, Arena *temp) {
    System &S = *PK.S;
    if (S.vt != SGTV_F32) HIP_TRY(upload(S.colscale, PK.colscale));
    if (S.format == SGTV_FORMAT_TILED) {
        if (int e = upload_tiled(S.fwd, PK.fwd)) return e;
        if (int e = upload_tiled(S.back, PK.back)) return e;
        HIP_TRY(S.fpart.alloc(sizeof(float) * PK.fpart_floats));
        HIP_TRY(S.bpart.alloc(sizeof(float) * PK.bpart_floats));
        if (int e = alloc_counters(c, S)) return e;
    } else {
        if (S.vt == SGTV_F32) {
            HIP_TRY(upload(S.rs_val, PK.rsv32));
            HIP_TRY(upload(S.cs_val, PK.csv32));
        } else {
            HIP_TRY(upload(S.rs_val, PK.rsv16));
            HIP_TRY(upload(S.cs_val, PK.csv16));
        }
        HIP_TRY(upload(S.rs_ptr, PK.rsp));
        HIP_TRY(upload(S.rs_idx, PK.rsi));
        HIP_TRY(upload(S.cs_ptr, PK.csp));
        HIP_TRY(upload(S.cs_idx, PK.csi));
    }
    HIP_TRY(upload(S.H, PK.H));
    HIP_TRY(upload(S.htab, PK.htab));
    if (S.wfull) HIP_TRY(upload(S.wbuf, PK.wf));
    return compute_sensitivity(c, S, temp);
}

// The sensitivity s = A^T 1 of a system whose arrays are on the device.
int compute_sensitivity(sgtv_ctx_s *c, System &S, Arena *temp) {
    HIP_TRY(S.sens.alloc(sizeof(float) * S.J));
    if (counting()) return SGTV_OK;
    // sensitivity s = A^T 1 with the stored (possibly quantised) values
    std::vector<float> ones(static_cast<size_t>(S.I + kVecPad), 1.0f);
    DBuf d_ones;
    {
        ArenaScope ts(temp, true);
        HIP_TRY(upload(d_ones, ones));
    }
    if (int e = back_project(S, d_ones.as<float>(), S.sens.as<float>(), c->stream)) return e;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SGTV_OK;
}

// FP64 partial sums the reductions of a system need.
int64_t partials_needed(const System &S) {
    const int64_t n1 = (S.n_rslices + 3) / 4;
    int sl = 0;
    while ((1 << sl) < S.Q && sl < 6) ++sl;
    const int64_t n2 = (S.S + (256 >> sl) - 1) / (256 >> sl);
    return std::max<int64_t>({n1, 6 * n2, 4096, 16});
}

int ensure_partials(sgtv_ctx_s *c) {
    const int64_t need = partials_needed(*c->sys);
    if (need > c->part_cap) {
        HIP_TRY(c->part.alloc(sizeof(double) * need));
        c->part_cap = need;
    }
    if (!c->red.p) HIP_TRY(c->red.alloc(sizeof(double) * 16));
    return SGTV_OK;
}

// Event bracket around one launch while profiling is on.
struct TimedLaunch {
    sgtv_ctx_s *c;
    int cls;
    hipEvent_t beg = nullptr;
    TimedLaunch(sgtv_ctx_s *ctx, int k) : c(ctx), cls(k) {
        if (c->profiling && hipEventCreate(&beg) == hipSuccess) (void)hipEventRecord(beg, c->stream);
    }
    ~TimedLaunch() {
        if (!beg) return;
        hipEvent_t end = nullptr;
        if (hipEventCreate(&end) == hipSuccess && hipEventRecord(end, c->stream) == hipSuccess)
            c->timed.push_back({cls, beg, end});
        else
            (void)hipEventDestroy(beg);
    }
};

int seg_log2_of(int Q) {
    int sl = 0;
    while ((1 << sl) < Q && sl < 6) ++sl;
    return sl;
}

// The fused image and split update applies: tiled format, a tile that fits
bool fused_ok(const sgtv_ctx_s *c) {
    const System &S = *c->sys;
    return c->fused && S.format == SGTV_FORMAT_TILED && S.fused_tw > 0 && S.fused_th > 0;
}

// One ADMM iteration (Eqs. 4-6) as a launch sequence on the context stream.
int step(sgtv_ctx_s *c) {
    const System &S = *c->sys;
    const sgtv::Weights w = S.weights();
    const float lam = static_cast<float>(c->rho);
    const float *scale = S.vt == SGTV_F32 ? nullptr : S.colscale.as<float>();
    float *gs_next = S.vt == SGTV_F32 ? nullptr : c->fs.as<float>();
    for (int sw = 0; sw < c->sweeps; ++sw) {
        const float *x = S.vt == SGTV_F32 ? c->f[c->fcur].as<float>() : c->fs.as<float>();
        if (S.format == SGTV_FORMAT_TILED) {
            const bool fused_last = sw + 1 == c->sweeps && fused_ok(c);
            if (c->epilogues) {
                // forward product and ratio in one launch
                TimedLaunch t(c, 0);
                const sgtv::RatioEpilogue E{S.fcount.as<uint32_t>(), c->y.as<float>(), c->r.as<float>(),
                                            c->ratio.as<float>()};
                HIP_TRY(sgtv::launch_tiled_ratio(S.fwd.map, S.vt, x, S.fpart.as<float>(), E, c->stream));
            } else {
                {
                    TimedLaunch t(c, 0);
                    HIP_TRY(sgtv::launch_tiled(S.fwd.map, S.vt, x, S.fpart.as<float>(), c->stream));
                }
                TimedLaunch t(c, 3);
                HIP_TRY(sgtv::launch_ratio_combine(S.fpart.as<float>(), S.fwd.map.ns, S.I, c->y.as<float>(),
                                                   c->r.as<float>(), c->ratio.as<float>(), nullptr, false,
                                                   c->stream, nullptr));
            }
            if (c->epilogues && !fused_last) {
                // back product and image update in one launch
                TimedLaunch t(c, 1);
                sgtv::UpdateEpilogue E{};
                E.count = S.bcount.as<uint32_t>();
                E.scale = scale;
                E.g = c->f[c->fcur].as<float>();
                E.g_next = c->f[c->fcur ^ 1].as<float>();
                E.gs_next = gs_next;
                E.v = c->v[c->vcur].as<float>();
                E.a = c->a[c->vcur].as<float>();
                E.sens = S.sens.as<float>();
                E.H = S.H.as<float>();
                E.htab = S.htab.as<float>();
                E.grid = S.grid;
                E.wts = w;
                E.lam = lam;
                HIP_TRY(sgtv::launch_tiled_update(S.back.map, S.vt, c->ratio.as<float>(), S.bpart.as<float>(), E,
                                                  c->grouping, c->stream));
                c->fcur ^= 1;
                continue;
            }
            {
                TimedLaunch t(c, 1);
                HIP_TRY(sgtv::launch_tiled(S.back.map, S.vt, c->ratio.as<float>(), S.bpart.as<float>(), c->stream));
            }
            if (fused_last) {
                // last sweep: the image update fused with the split and dual update
                TimedLaunch t(c, 4);
                sgtv::FusedUpdate A{};
                A.part = S.bpart.as<float>();
                A.ns = S.back.map.ns;
                A.scale = scale;
                A.g = c->f[c->fcur].as<float>();
                A.g_next = c->f[c->fcur ^ 1].as<float>();
                A.gs_next = gs_next;
                A.v_old = c->v[c->vcur].as<float>();
                A.a_old = c->a[c->vcur].as<float>();
                A.v_new = c->v[c->vcur ^ 1].as<float>();
                A.a_new = c->a[c->vcur ^ 1].as<float>();
                A.sens = S.sens.as<float>();
                A.H = S.H.as<float>();
                A.htab = S.htab.as<float>();
                A.grid = S.grid;
                A.wts = w;
                A.lam = lam;
                A.thr = static_cast<float>(c->beta / c->rho);
                A.tw = S.fused_tw;
                A.th = S.fused_th;
                A.tiles_x = (S.nx + S.fused_tw - 1) / S.fused_tw;
                A.seg_log2 = seg_log2_of(S.Q);
                HIP_TRY(sgtv::launch_update_fused(A, c->grouping, S.fused_threads, c->stream));
                c->fcur ^= 1;
                c->vcur ^= 1;
                c->k += 1;
                return SGTV_OK;
            }
            {
                TimedLaunch t(c, 4);
                HIP_TRY(sgtv::launch_voxel_update(S.bpart.as<float>(), S.back.map.ns, scale,
                                                  c->f[c->fcur].as<float>(), c->f[c->fcur ^ 1].as<float>(),
                                                  gs_next, c->v[c->vcur].as<float>(), c->a[c->vcur].as<float>(),
                                                  S.sens.as<float>(), S.H.as<float>(), S.htab.as<float>(), S.grid,
                                                  w, c->grouping, lam, c->stream));
            }
        } else {
            {
                TimedLaunch t(c, 0);
                HIP_TRY(sgtv::launch_forward_ratio(S.rows(), S.vt, x, c->y.as<float>(), c->r.as<float>(),
                                                   c->ratio.as<float>(), nullptr, false, c->stream, nullptr));
            }
            TimedLaunch t(c, 1);
            HIP_TRY(sgtv::launch_back_update(S.cols(), S.vt, c->ratio.as<float>(), c->f[c->fcur].as<float>(),
                                             c->f[c->fcur ^ 1].as<float>(), c->fs.as<float>(),
                                             c->v[c->vcur].as<float>(), c->a[c->vcur].as<float>(),
                                             S.sens.as<float>(), S.H.as<float>(), S.grid, w,
                                             c->grouping, lam, c->stream));
        }
        c->fcur ^= 1;
    }
    TimedLaunch t(c, 2);
    HIP_TRY(sgtv::launch_split_update(c->f[c->fcur].as<float>(), c->v[c->vcur].as<float>(),
                                      c->a[c->vcur].as<float>(), c->v[c->vcur ^ 1].as<float>(),
                                      c->a[c->vcur ^ 1].as<float>(), S.grid, w, c->grouping,
                                      static_cast<float>(c->beta / c->rho), c->stream));
    c->vcur ^= 1;
    c->k += 1;
    return SGTV_OK;
}

// Argument checks of sgtv_set_system / sgtv_plan_system that need no data.
int check_system_args(int64_t I, int32_t ny, int32_t nx, int32_t Q, const int64_t *row_ptr, const int32_t *col_idx,
                      const float *val, int64_t nnz, int storage_dtype, const float *w, int64_t w_len,
                      int mem_kind) {
    if (int e = check_mem_kind(mem_kind)) return e;
    if (I < 1 || ny < 1 || nx < 1 || Q < 1) return fail(SGTV_ESHAPE, "I, ny, nx and Q must be >= 1");
    if (nnz < 0 || nnz >= (int64_t(1) << 31)) return fail(SGTV_ESHAPE, "nnz must be in [0, 2^31)");
    const int64_t J = static_cast<int64_t>(ny) * nx * Q;
    if (J >= (int64_t(1) << 31)) return fail(SGTV_ESHAPE, "J = ny*nx*Q must be below 2^31");
    if (I >= (int64_t(1) << 31)) return fail(SGTV_ESHAPE, "I must be below 2^31");
    if (storage_dtype != SGTV_F32 && storage_dtype != SGTV_BF16 && storage_dtype != SGTV_F16)
        return fail(SGTV_EINVAL, "unknown storage dtype");
    if (!row_ptr || (nnz > 0 && (!col_idx || !val))) return fail(SGTV_EINVAL, "NULL matrix array");
    if (w && w_len != 4 && w_len != 4 * J) return fail(SGTV_ESHAPE, "w_len must be 4 or 4*J");
    if (!w && w_len != 0) return fail(SGTV_ESHAPE, "w is NULL but w_len is not 0");
    return SGTV_OK;
}

// Replace the context's system (may be null) and drop its data and state.
void install_system(sgtv_ctx_s *ctx, std::unique_ptr<System> S) {
    drop_graphs(ctx);
    ctx->sys = std::move(S);
    ctx->has_data = false;
    ctx->y.release(); ctx->r.release(); ctx->ratio.release();
    for (int b = 0; b < 2; ++b) { ctx->f[b].release(); ctx->v[b].release(); ctx->a[b].release(); }
    ctx->fs.release();
    ctx->part_cap = 0;
    ctx->part.release();
    ctx->red.release();
}

// The sections of the context's workspace, or null when the library
// allocates the context's memory itself.
Arena *ws_section(sgtv_ctx_s *c, Arena Workspace::*sec) { return c->ws.base ? &(c->ws.*sec) : nullptr; }

}  // namespace

extern "C" {

const char *sgtv_last_error(void) { return g_err.c_str(); }

const char *sgtv_version(void) { return "sgtv 0.2 (gfx950; tiled and sliced-ELL formats; FP32, BF16, FP16 values)"; }

int sgtv_create(sgtv_ctx *out, int device, void *hip_stream) {
    if (!out) return fail(SGTV_EINVAL, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(SGTV_EINVAL, "device index out of range");
    {
        // set-up of the static device buffer on this device (once per device)
        DeviceGuard g(device);
        if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
        float *sp = nullptr;
        HIP_TRY(scratch_address(device, &sp));
    }
    try {
        auto c = new sgtv_ctx_s();
        c->device = device;
        c->stream = static_cast<hipStream_t>(hip_stream);
        *out = c;
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

void sgtv_destroy(sgtv_ctx ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (auto &t : ctx->timed) {
        (void)hipEventDestroy(t.beg);
        (void)hipEventDestroy(t.end);
    }
    drop_graphs(ctx);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
}

int sgtv_set_system(sgtv_ctx ctx, int64_t I, int32_t ny, int32_t nx, int32_t Q,
                    const int64_t *row_ptr, const int32_t *col_idx, const float *val,
                    int64_t nnz, int storage_dtype, const float *w, int64_t w_len, int mem_kind) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (int e = check_system_args(I, ny, nx, Q, row_ptr, col_idx, val, nnz, storage_dtype, w, w_len, mem_kind))
        return e;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    try {
        Packed PK;
        if (int e = pack_system(ctx, PK, I, ny, nx, Q, row_ptr, col_idx, val, nnz, storage_dtype, w, w_len,
                                mem_kind))
            return e;
        if (int e = upload_system(ctx, PK, nullptr)) return e;
        // commit: from now on the library allocates the context's memory itself
        install_system(ctx, std::move(PK.S));
        ctx->ws = Workspace{};
        ctx->pending.reset();
        if (int e = ensure_partials(ctx)) return e;
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

namespace {

// Bytes of the sections of a workspace: data, state and temporaries (the
// system section is counted by a dry upload).
size_t data_section_bytes(const System &S) {
    return align_up(sizeof(float) * (S.I + kVecPad)) + align_up(sizeof(float) * S.I) +
           align_up(sizeof(float) * (S.I + kVecPad));
}

size_t state_section_bytes(const System &S) {
    // f and v double buffered, a sized for either grouping (at most J), the scaled copy
    return 2 * align_up(sizeof(float) * (S.J + kVecPad)) + 2 * align_up(sizeof(float) * S.J * 4) +
           2 * align_up(sizeof(float) * S.J) + align_up(sizeof(float) * (S.J + kVecPad));
}

size_t temp_section_bytes(const System &S) {
    const size_t j4 = align_up(sizeof(float) * S.J), v4 = align_up(sizeof(float) * S.J * 4);
    return std::max({align_up(sizeof(float) * (S.I + kVecPad)),   // ones of the sensitivity
                     2 * v4,                                       // d and c of get_split
                     j4 + v4 + j4,                                 // f, v, a of set_state
                     2 * j4});                                     // backprojection
}

}  // namespace

int sgtv_plan_system(sgtv_ctx ctx, int64_t I, int32_t ny, int32_t nx, int32_t Q, const int64_t *row_ptr,
                     const int32_t *col_idx, const float *val, int64_t nnz, int storage_dtype, const float *w,
                     int64_t w_len, int mem_kind, int64_t *bytes) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (!bytes) return fail(SGTV_EINVAL, "bytes is NULL");
    if (int e = check_system_args(I, ny, nx, Q, row_ptr, col_idx, val, nnz, storage_dtype, w, w_len, mem_kind))
        return e;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
    try {
        auto PK = std::make_unique<Packed>();
        if (int e = pack_system(ctx, *PK, I, ny, nx, Q, row_ptr, col_idx, val, nnz, storage_dtype, w, w_len,
                                mem_kind))
            return e;
        // the system section: the same allocations as the upload, counted
        Arena cnt;
        cnt.count = true;
        {
            ArenaScope sc(&cnt, true);
            if (int e = upload_system(ctx, *PK, nullptr)) return e;
            DBuf part, red;
            HIP_TRY(part.alloc(sizeof(double) * partials_needed(*PK->S)));
            HIP_TRY(red.alloc(sizeof(double) * 16));
        }
        const System &S = *PK->S;
        const size_t sec[4] = {align_up(cnt.used), data_section_bytes(S), state_section_bytes(S),
                               temp_section_bytes(S)};
        ctx->pending = std::move(PK);
        for (int k = 0; k < 4; ++k) ctx->pending_sections[k] = sec[k];
        ctx->pending_bytes = static_cast<int64_t>(sec[0] + sec[1] + sec[2] + sec[3]);
        *bytes = ctx->pending_bytes;
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

int sgtv_commit_system(sgtv_ctx ctx, void *workspace, int64_t bytes) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (!ctx->pending) return fail(SGTV_ESTATE, "no planned system (call sgtv_plan_system first)");
    if (!workspace) return fail(SGTV_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(SGTV_EINVAL, "workspace must be aligned to 256 bytes");
    if (bytes < ctx->pending_bytes)
        return fail(SGTV_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes; the planned system needs " +
                                     std::to_string(ctx->pending_bytes));
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    try {
        Workspace ws;
        ws.base = static_cast<char *>(workspace);
        ws.size = static_cast<size_t>(bytes);
        Arena *sec[4] = {&ws.sys, &ws.data, &ws.state, &ws.temp};
        size_t off = 0;
        for (int k = 0; k < 4; ++k) {
            sec[k]->base = ws.base + off;
            sec[k]->cap = ctx->pending_sections[k];
            off += ctx->pending_sections[k];
        }
        // the old system and state go first (their memory may be reused)
        drop_graphs(ctx);
        install_system(ctx, nullptr);
        ctx->ws = ws;
        Packed &PK = *ctx->pending;
        {
            ArenaScope sc(&ctx->ws.sys, true);
            if (int e = upload_system(ctx, PK, &ctx->ws.temp)) {
                ctx->ws = Workspace{};
                return e;
            }
            install_system(ctx, std::move(PK.S));
            if (int e = ensure_partials(ctx)) return e;
        }
        ctx->pending.reset();
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

}  // extern "C"

namespace {

// File of a packed system (sgtv_save_system / sgtv_load_system):
//   FileHead, SysMeta, the row permutation (I int64), one ArrayRec per device
//   array, a 64-bit hash of all of these; then the arrays' bytes, one after
//   the other (every byte of the file is covered by a hash).
// Arrays move in chunks of kIoChunk bytes through pinned staging buffers, one
// per host thread, and every chunk is hashed on the way; an array's hash
// folds its chunk hashes in order, so it does not depend on the threads.
constexpr char kSysMagic[8] = {'S', 'G', 'T', 'V', 'S', 'Y', 'S', '1'};
constexpr uint32_t kSysVersion = 3;
constexpr size_t kIoChunk = size_t(8) << 20;
constexpr int kSysArrays = 20;

struct FileHead {
    char magic[8];
    uint32_t version, meta_bytes, map_bytes, n_arrays;
    int64_t n_perm;
};

struct SysMeta {
    int64_t I, J, S, nnz;
    int32_t ny, nx, Q, vt, format, wfull, fused_tw, fused_th, fused_threads, pad_;
    sgtv_schedule sched;
    float w4[4];
    int64_t n_rslices, n_cslices, fpart_bytes, bpart_bytes;
    sgtv::TileMap fwd, back;   // the pointers in it are not used
};

struct ArrayRec {
    int64_t offset, bytes;
    uint64_t hash;
    int32_t present, pad_;
};

constexpr uint64_t kHashBasis = 1469598103934665603ull, kHashPrime = 1099511628211ull;

uint64_t hash_step(uint64_t h, uint64_t x) { return (((h << 23) | (h >> 41)) ^ x) * kHashPrime; }

// Four interleaved lanes over 8-byte words, the tail and the length last.
uint64_t chunk_hash(const unsigned char *p, size_t n) {
    uint64_t h[4] = {kHashBasis, kHashBasis + 1, kHashBasis + 2, kHashBasis + 3};
    const size_t nw = n / 8;
    size_t k = 0;
    for (; k + 4 <= nw; k += 4)
        for (int l = 0; l < 4; ++l) {
            uint64_t x;
            std::memcpy(&x, p + 8 * (k + l), 8);
            h[l] = hash_step(h[l], x);
        }
    for (; k < nw; ++k) {
        uint64_t x;
        std::memcpy(&x, p + 8 * k, 8);
        h[0] = hash_step(h[0], x);
    }
    uint64_t tail = 0;
    std::memcpy(&tail, p + 8 * nw, n - 8 * nw);
    uint64_t r = hash_step(h[0], h[1]);
    r = hash_step(r, h[2]);
    r = hash_step(r, h[3]);
    r = hash_step(r, tail);
    return hash_step(r, static_cast<uint64_t>(n));
}

// The device arrays of a system in file order.
template <class F>
void each_array(System &S, F fn) {
    for (DBuf *d : {&S.colscale, &S.H, &S.htab, &S.wbuf, &S.fwd.pk, &S.fwd.val, &S.fwd.goff, &S.fwd.poff,
                    &S.fwd.slot, &S.back.pk, &S.back.val, &S.back.goff, &S.back.poff, &S.back.slot, &S.rs_ptr,
                    &S.rs_idx, &S.rs_val, &S.cs_ptr, &S.cs_idx, &S.cs_val})
        fn(*d);
}

struct FileCloser {
    int fd = -1;
    ~FileCloser() {
        if (fd >= 0) ::close(fd);
    }
};

// Moves the arrays between the device and the file in chunks, on the host
// threads, each with its own pinned staging buffer; fills chunk hashes (in
// order per array).  to_file: device -> file, else file -> device.
int move_arrays(int device, int fd, std::vector<DBuf *> &bufs, const std::vector<ArrayRec> &rec, bool to_file,
                std::vector<uint64_t> &hashes) {
    struct Item {
        int a;
        int64_t off;
        size_t n;
    };
    std::vector<Item> items;
    std::vector<size_t> first(bufs.size() + 1, 0);
    for (size_t a = 0; a < bufs.size(); ++a) {
        first[a] = items.size();
        for (int64_t off = 0; off < rec[a].bytes; off += static_cast<int64_t>(kIoChunk))
            items.push_back({static_cast<int>(a), off,
                             static_cast<size_t>(std::min<int64_t>(kIoChunk, rec[a].bytes - off))});
    }
    first[bufs.size()] = items.size();
    std::vector<uint64_t> ch(items.size(), 0);
    std::atomic<int> status{SGTV_OK};
    std::mutex msg_mu;
    std::string msg;
    auto set_error = [&](int code, const std::string &m) {
        int ok = SGTV_OK;
        if (status.compare_exchange_strong(ok, code)) {
            std::lock_guard<std::mutex> lk(msg_mu);
            msg = m;
        }
    };
    on_threads(static_cast<int64_t>(items.size()), [&](int64_t me, int64_t step) {
        if (hipSetDevice(device) != hipSuccess) {
            set_error(SGTV_EDEVICE, "cannot select device");
            return;
        }
        void *stage = nullptr;
        if (hipHostMalloc(&stage, kIoChunk) != hipSuccess) {
            set_error(SGTV_ENOMEM, "pinned staging buffer of 8 MiB");
            return;
        }
        unsigned char *buf = static_cast<unsigned char *>(stage);
        for (int64_t k = me; k < static_cast<int64_t>(items.size()) && status.load() == SGTV_OK; k += step) {
            const Item &it = items[k];
            char *dev = static_cast<char *>(bufs[it.a]->p) + it.off;
            const off_t at = static_cast<off_t>(rec[it.a].offset + it.off);
            if (to_file) {
                hipError_t e = hipMemcpy(buf, dev, it.n, hipMemcpyDeviceToHost);
                if (e != hipSuccess) {
                    set_error(SGTV_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
                    break;
                }
                ch[k] = chunk_hash(buf, it.n);
                for (size_t done = 0; done < it.n;) {
                    const ssize_t w = ::pwrite(fd, buf + done, it.n - done, at + static_cast<off_t>(done));
                    if (w <= 0) {
                        set_error(SGTV_EINVAL, "writing the system file failed");
                        break;
                    }
                    done += static_cast<size_t>(w);
                }
            } else {
                size_t done = 0;
                while (done < it.n) {
                    const ssize_t r = ::pread(fd, buf + done, it.n - done, at + static_cast<off_t>(done));
                    if (r <= 0) break;
                    done += static_cast<size_t>(r);
                }
                if (done != it.n) {
                    set_error(SGTV_EINVAL, "the system file is truncated");
                    break;
                }
                ch[k] = chunk_hash(buf, it.n);
                hipError_t e = hipMemcpy(dev, buf, it.n, hipMemcpyHostToDevice);
                if (e != hipSuccess) {
                    set_error(SGTV_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
                    break;
                }
            }
        }
        (void)hipHostFree(stage);
    });
    if (status.load() != SGTV_OK) return fail(status.load(), msg);
    hashes.assign(bufs.size(), 0);
    for (size_t a = 0; a < bufs.size(); ++a) {
        uint64_t h = kHashBasis;
        for (size_t k = first[a]; k < first[a + 1]; ++k) h = hash_step(h, ch[k]);
        hashes[a] = hash_step(h, static_cast<uint64_t>(rec[a].bytes));
    }
    return SGTV_OK;
}

std::vector<char> head_bytes(const FileHead &fh, const SysMeta &m, const std::vector<int64_t> &perm,
                             const std::vector<ArrayRec> &rec) {
    std::vector<char> b(sizeof(fh) + sizeof(m) + sizeof(int64_t) * perm.size() + sizeof(ArrayRec) * rec.size());
    char *p = b.data();
    std::memcpy(p, &fh, sizeof(fh)); p += sizeof(fh);
    std::memcpy(p, &m, sizeof(m)); p += sizeof(m);
    if (!perm.empty()) std::memcpy(p, perm.data(), sizeof(int64_t) * perm.size());
    p += sizeof(int64_t) * perm.size();
    std::memcpy(p, rec.data(), sizeof(ArrayRec) * rec.size());
    return b;
}

}  // namespace

extern "C" {

int sgtv_save_system(sgtv_ctx ctx, const char *path) {
    if (!ctx || !path) return fail(SGTV_EINVAL, "null argument");
    if (!ctx->sys) return fail(SGTV_ESTATE, "no system set");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    try {
        System &S = *ctx->sys;
        SysMeta m{};
        m.I = S.I; m.J = S.J; m.S = S.S; m.nnz = S.nnz;
        m.ny = S.ny; m.nx = S.nx; m.Q = S.Q; m.vt = S.vt; m.format = S.format; m.wfull = S.wfull ? 1 : 0;
        m.fused_tw = S.fused_tw; m.fused_th = S.fused_th; m.fused_threads = S.fused_threads;
        m.sched = S.sched;
        for (int p = 0; p < 4; ++p) m.w4[p] = S.w4[p];
        m.n_rslices = S.n_rslices; m.n_cslices = S.n_cslices;
        m.fpart_bytes = static_cast<int64_t>(S.fpart.bytes);
        m.bpart_bytes = static_cast<int64_t>(S.bpart.bytes);
        m.fwd = S.fwd.map;
        m.back = S.back.map;
        FileHead fh{};
        std::memcpy(fh.magic, kSysMagic, 8);
        fh.version = kSysVersion;
        fh.meta_bytes = sizeof(SysMeta);
        fh.map_bytes = sizeof(sgtv::TileMap);
        fh.n_arrays = kSysArrays;
        fh.n_perm = static_cast<int64_t>(S.perm.size());
        std::vector<DBuf *> bufs;
        each_array(S, [&](DBuf &d) { bufs.push_back(&d); });
        std::vector<ArrayRec> rec(bufs.size());
        int64_t off = static_cast<int64_t>(head_bytes(fh, m, S.perm, rec).size() + 8);
        for (size_t a = 0; a < bufs.size(); ++a) {
            rec[a].offset = off;
            rec[a].bytes = static_cast<int64_t>(bufs[a]->bytes);
            rec[a].present = bufs[a]->p != nullptr;
            off += rec[a].bytes;
        }
        FileCloser fc;
        fc.fd = ::open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
        if (fc.fd < 0) return fail(SGTV_EINVAL, std::string("cannot open ") + path + " for writing");
        std::vector<uint64_t> hashes;
        if (int e = move_arrays(ctx->device, fc.fd, bufs, rec, true, hashes)) return e;
        for (size_t a = 0; a < bufs.size(); ++a) rec[a].hash = hashes[a];
        std::vector<char> head = head_bytes(fh, m, S.perm, rec);
        const uint64_t hh = chunk_hash(reinterpret_cast<const unsigned char *>(head.data()), head.size());
        head.resize(head.size() + 8);
        std::memcpy(head.data() + head.size() - 8, &hh, 8);
        if (::pwrite(fc.fd, head.data(), head.size(), 0) != static_cast<ssize_t>(head.size()) ||
            ::ftruncate(fc.fd, static_cast<off_t>(off)) != 0)
            return fail(SGTV_EINVAL, std::string("writing ") + path + " failed");
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

int sgtv_load_system(sgtv_ctx ctx, const char *path) {
    if (!ctx || !path) return fail(SGTV_EINVAL, "null argument");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    try {
        FileCloser fc;
        fc.fd = ::open(path, O_RDONLY);
        if (fc.fd < 0) return fail(SGTV_EINVAL, std::string("cannot open ") + path);
        struct stat st{};
        if (::fstat(fc.fd, &st) != 0) return fail(SGTV_EINVAL, std::string("cannot stat ") + path);
        const int64_t fsize = static_cast<int64_t>(st.st_size);
        const std::string bad = std::string(path) + " is not a system file of this library version";
        FileHead fh{};
        if (::pread(fc.fd, &fh, sizeof(fh), 0) != static_cast<ssize_t>(sizeof(fh)) ||
            std::memcmp(fh.magic, kSysMagic, 8) != 0 || fh.version != kSysVersion ||
            fh.meta_bytes != sizeof(SysMeta) || fh.map_bytes != sizeof(sgtv::TileMap) ||
            fh.n_arrays != kSysArrays || fh.n_perm < 0 || fh.n_perm > (int64_t(1) << 31))
            return fail(SGTV_EINVAL, bad);
        const size_t hb = sizeof(fh) + sizeof(SysMeta) + sizeof(int64_t) * static_cast<size_t>(fh.n_perm) +
                          sizeof(ArrayRec) * kSysArrays;
        if (static_cast<int64_t>(hb + 8) > fsize) return fail(SGTV_EINVAL, std::string(path) + " is truncated");
        std::vector<char> head(hb + 8);
        if (::pread(fc.fd, head.data(), head.size(), 0) != static_cast<ssize_t>(head.size()))
            return fail(SGTV_EINVAL, std::string(path) + " is truncated");
        uint64_t hh;
        std::memcpy(&hh, head.data() + hb, 8);
        if (hh != chunk_hash(reinterpret_cast<const unsigned char *>(head.data()), hb))
            return fail(SGTV_EINVAL, std::string(path) + ": damaged header");
        SysMeta m;
        const char *p = head.data() + sizeof(fh);
        std::memcpy(&m, p, sizeof(m)); p += sizeof(m);
        auto Sp = std::make_unique<System>();
        System &S = *Sp;
        S.perm.resize(static_cast<size_t>(fh.n_perm));
        if (fh.n_perm) std::memcpy(S.perm.data(), p, sizeof(int64_t) * S.perm.size());
        p += sizeof(int64_t) * S.perm.size();
        std::vector<ArrayRec> rec(kSysArrays);
        std::memcpy(rec.data(), p, sizeof(ArrayRec) * kSysArrays);
        // the description must be one the packer makes
        const bool shape_ok = m.I >= 1 && m.ny >= 1 && m.nx >= 1 && m.Q >= 1 && m.S == int64_t(m.ny) * m.nx &&
                              m.J == m.S * m.Q && m.J < (int64_t(1) << 31) && m.I < (int64_t(1) << 31) &&
                              (m.vt == SGTV_F32 || m.vt == SGTV_BF16 || m.vt == SGTV_F16) &&
                              (m.format == SGTV_FORMAT_TILED || m.format == SGTV_FORMAT_SELL) &&
                              fh.n_perm == m.I && m.fpart_bytes >= 0 && m.bpart_bytes >= 0;
        if (!shape_ok) return fail(SGTV_EINVAL, std::string(path) + ": inconsistent system description");
        S.I = m.I; S.J = m.J; S.S = m.S; S.nnz = m.nnz;
        S.ny = m.ny; S.nx = m.nx; S.Q = m.Q; S.vt = m.vt; S.format = m.format; S.wfull = m.wfull != 0;
        S.fused_tw = m.fused_tw; S.fused_th = m.fused_th; S.fused_threads = m.fused_threads;
        S.sched = m.sched;
        for (int q = 0; q < 4; ++q) S.w4[q] = m.w4[q];
        S.grid = sgtv::Grid{S.ny, S.nx, S.Q, S.S, S.J};
        S.n_rslices = m.n_rslices; S.n_cslices = m.n_cslices;
        S.fwd.map = m.fwd;
        S.back.map = m.back;
        std::vector<DBuf *> bufs;
        each_array(S, [&](DBuf &d) { bufs.push_back(&d); });
        for (const ArrayRec &r : rec)
            if (r.bytes < 0 || r.offset < static_cast<int64_t>(hb) || r.offset > fsize || r.bytes > fsize - r.offset ||
                (r.bytes > 0 && !r.present))
                return fail(SGTV_EINVAL, std::string(path) + " is truncated or inconsistent");
        // the arrays the kernels index must have the sizes the description implies
        auto rec_of = [&](const DBuf &d) -> const ArrayRec & {
            for (size_t a = 0; a < bufs.size(); ++a)
                if (bufs[a] == &d) return rec[a];
            return rec[0];
        };
        bool sizes_ok = rec_of(S.H).bytes == 4 * S.J && rec_of(S.htab).bytes == 64 &&
                        (S.vt == SGTV_F32 || rec_of(S.colscale).bytes == 4 * S.J) &&
                        (!S.wfull || rec_of(S.wbuf).bytes == 16 * S.J);
        if (S.format == SGTV_FORMAT_TILED)
            for (const Tiled *T : {&S.fwd, &S.back}) {
                const sgtv::TileMap &t = T->map;
                const int64_t n_lists = t.n_rb * static_cast<int64_t>(t.ns) * t.cbs_max * t.waves;
                sizes_ok = sizes_ok && t.ns >= 1 && t.ns <= sgtv::kMaxSlabs && n_lists >= 0 &&
                           rec_of(T->goff).bytes == 4 * (n_lists + 1);
            }
        if (!sizes_ok) return fail(SGTV_EINVAL, std::string(path) + ": inconsistent arrays");
        for (size_t a = 0; a < bufs.size(); ++a)
            if (rec[a].present) HIP_TRY(bufs[a]->alloc(static_cast<size_t>(rec[a].bytes)));
        std::vector<uint64_t> hashes;
        if (int e = move_arrays(ctx->device, fc.fd, bufs, rec, false, hashes)) return e;
        for (size_t a = 0; a < bufs.size(); ++a)
            if (hashes[a] != rec[a].hash) return fail(SGTV_EINVAL, std::string(path) + ": damaged array data");
        if (S.format == SGTV_FORMAT_TILED) {
            point_tiled(S.fwd);
            point_tiled(S.back);
            HIP_TRY(S.fpart.alloc(static_cast<size_t>(m.fpart_bytes)));
            HIP_TRY(S.bpart.alloc(static_cast<size_t>(m.bpart_bytes)));
            if (int e = alloc_counters(ctx, S)) return e;
        }
        if (int e = compute_sensitivity(ctx, S, nullptr)) return e;
        install_system(ctx, std::move(Sp));
        ctx->ws = Workspace{};
        ctx->pending.reset();
        if (int e = ensure_partials(ctx)) return e;
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

int sgtv_set_data(sgtv_ctx ctx, const float *y, const float *r, double beta, double rho,
                  int sweeps, int mem_kind) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (!ctx->sys) return fail(SGTV_ESTATE, "no system set (call sgtv_set_system first)");
    if (int e = check_mem_kind(mem_kind)) return e;
    if (!y || !r) return fail(SGTV_EINVAL, "NULL y or r");
    if (!(std::isfinite(beta) && beta >= 0.0)) return fail(SGTV_EINVAL, "beta must be finite and >= 0");
    if (!(std::isfinite(rho) && rho > 0.0)) return fail(SGTV_EINVAL, "rho must be finite and > 0");
    if (sweeps < 1) return fail(SGTV_EINVAL, "sweeps must be >= 1");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    try {
        const System &S = *ctx->sys;
        std::vector<float> hy, hr;
        HIP_TRY(fetch(hy, y, S.I, mem_kind));
        HIP_TRY(fetch(hr, r, S.I, mem_kind));
        for (int64_t i = 0; i < S.I; ++i) {
            if (!finite_nonneg(hy[i])) return fail(SGTV_EINVAL, "y has a negative or non-finite value at " + std::to_string(i));
            if (!(std::isfinite(hr[i]) && hr[i] > 0.0f)) return fail(SGTV_EINVAL, "r must be finite and > 0 (index " + std::to_string(i) + ")");
        }
        // vectors gathered by the tiled products carry kVecPad spare floats
        std::vector<float> py(static_cast<size_t>(S.I + kVecPad), 0.0f), pr(static_cast<size_t>(S.I), 0.0f);
        for (int64_t i = 0; i < S.I; ++i) { py[i] = hy[S.perm[i]]; pr[i] = hr[S.perm[i]]; }
        DBuf dy, dr, dratio;
        {
            // in a workspace the data section is refilled (the old y, r and
            // ratio are replaced in place; the host checks above have passed)
            ArenaScope sc(ws_section(ctx, &Workspace::data), true);
            HIP_TRY(upload(dy, py));
            HIP_TRY(upload(dr, pr));
            HIP_TRY(dratio.alloc(sizeof(float) * (S.I + kVecPad)));
        }
        drop_graphs(ctx);
        ctx->y = std::move(dy);
        ctx->r = std::move(dr);
        ctx->ratio = std::move(dratio);
        ctx->beta = beta;
        ctx->rho = rho;
        ctx->sweeps = sweeps;
        if (!ctx->f[0].p || ctx->a[0].bytes != sizeof(float) * n_groups(ctx)) {
            ArenaScope sc(ws_section(ctx, &Workspace::state), true);
            if (int e = alloc_state(ctx)) return e;
        }
        ctx->has_data = true;
        if (int e = uniform_start(ctx)) return e;
        if (int e = refresh_scaled(ctx)) return e;
        if (int e = clear_split(ctx)) return e;
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

int sgtv_set_grouping(sgtv_ctx ctx, int grouping) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (grouping != SGTV_GROUP_SPECTRAL && grouping != SGTV_GROUP_STANDARD)
        return fail(SGTV_EINVAL, "unknown grouping");
    if (grouping == ctx->grouping) {
        if (ctx->sys && ctx->has_data) {
            DeviceGuard g(ctx->device);
            return clear_split(ctx);
        }
        return SGTV_OK;
    }
    DeviceGuard g(ctx->device);
    drop_graphs(ctx);
    const int old = ctx->grouping;
    ctx->grouping = grouping;
    if (ctx->sys && ctx->has_data) {
        // keep f, resize (v, a) storage for the new group count
        DBuf keep_f;
        {
            ArenaScope sc(ws_section(ctx, &Workspace::temp), true);
            HIP_TRY(keep_f.alloc(sizeof(float) * ctx->sys->J));
        }
        HIP_TRY(hipMemcpyAsync(keep_f.p, ctx->f[ctx->fcur].p, sizeof(float) * ctx->sys->J,
                               hipMemcpyDeviceToDevice, ctx->stream));
        {
            ArenaScope sc(ws_section(ctx, &Workspace::state), true);
            if (int e = alloc_state(ctx)) { ctx->grouping = old; return e; }
        }
        HIP_TRY(hipMemcpyAsync(ctx->f[0].p, keep_f.p, sizeof(float) * ctx->sys->J,
                               hipMemcpyDeviceToDevice, ctx->stream));
        ctx->fcur = 0;
        if (int e = refresh_scaled(ctx)) return e;
        if (int e = clear_split(ctx)) return e;
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    return SGTV_OK;
}

int sgtv_set_init(sgtv_ctx ctx, const float *x0, int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    DeviceGuard g(ctx->device);
    try {
        const System &S = *ctx->sys;
        drop_graphs(ctx);
        if (x0) {
            DBuf staged;
            ArenaScope sc(ws_section(ctx, &Workspace::temp), true);
            if (int e = stage_floats(staged, x0, S.J, mem_kind, ctx->stream, finite_nonneg, "x0"))
                return e;
            HIP_TRY(hipMemcpyAsync(ctx->f[0].p, staged.p, sizeof(float) * S.J,
                                   hipMemcpyDeviceToDevice, ctx->stream));
            ctx->fcur = 0;
        } else {
            if (int e = uniform_start(ctx)) return e;
        }
        if (int e = refresh_scaled(ctx)) return e;
        if (int e = clear_split(ctx)) return e;
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

int sgtv_set_init_dual(sgtv_ctx ctx, const float *x0, int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    if (!x0) return fail(SGTV_EINVAL, "x0 is NULL");
    DeviceGuard g(ctx->device);
    try {
        const System &S = *ctx->sys;
        DBuf staged;
        ArenaScope sc(ws_section(ctx, &Workspace::temp), true);
        if (int e = stage_floats(staged, x0, S.J, mem_kind, ctx->stream, finite_nonneg, "x0")) return e;
        drop_graphs(ctx);
        HIP_TRY(hipMemcpyAsync(ctx->f[0].p, staged.p, sizeof(float) * S.J, hipMemcpyDeviceToDevice, ctx->stream));
        ctx->fcur = 0;
        ctx->vcur = 0;
        HIP_TRY(sgtv::launch_consistent_split(ctx->f[0].as<float>(), ctx->v[0].as<float>(), ctx->a[0].as<float>(),
                                              S.grid, S.weights(), ctx->grouping,
                                              static_cast<float>(ctx->beta / ctx->rho), ctx->stream));
        HIP_TRY(hipMemcpyAsync(ctx->v[1].p, ctx->v[0].p, sizeof(float) * S.J * 4, hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(ctx->a[1].p, ctx->a[0].p, sizeof(float) * n_groups(ctx), hipMemcpyDeviceToDevice, ctx->stream));
        ctx->k = 0;
        if (int e = refresh_scaled(ctx)) return e;
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

namespace {

// The graph of n_iters iterations from the current buffer parity: found in the
// cache or captured (not run) and instantiated.  The state is left unchanged.
int context_graph(sgtv_ctx ctx, int n_iters, Context::Graph *out) {
    for (auto &gr : ctx->graphs)
        if (gr.n == n_iters && gr.fcur == ctx->fcur && gr.vcur == ctx->vcur) {
            *out = gr;
            return SGTV_OK;
        }
    // capture the launch sequence on the context's own stream
    if (!ctx->cap) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    const int f0 = ctx->fcur, v0 = ctx->vcur;
    const int64_t k0 = ctx->k;
    hipStream_t user = ctx->stream;
    ctx->stream = ctx->cap;
    hipError_t e = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed);
    int status = e == hipSuccess ? SGTV_OK : hip_fail(e, "hipStreamBeginCapture");
    for (int it = 0; it < n_iters && status == SGTV_OK && e == hipSuccess; ++it) status = step(ctx);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) {
        hipError_t e2 = hipStreamEndCapture(ctx->cap, &graph);
        if (status == SGTV_OK && e2 != hipSuccess) status = hip_fail(e2, "hipStreamEndCapture");
    }
    ctx->stream = user;
    Context::Graph gr{n_iters, f0, v0, ctx->fcur, ctx->vcur, nullptr};
    ctx->fcur = f0;
    ctx->vcur = v0;
    ctx->k = k0;
    if (status == SGTV_OK) {
        hipError_t e3 = hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0);
        if (e3 != hipSuccess) status = hip_fail(e3, "hipGraphInstantiate");
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (status != SGTV_OK) return status;
    if (ctx->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(gr);
    *out = gr;
    return SGTV_OK;
}

}  // namespace

int sgtv_iterate(sgtv_ctx ctx, int n_iters) {
    if (int e = check_ready(ctx)) return e;
    if (n_iters < 0) return fail(SGTV_EINVAL, "n_iters must be >= 0");
    DeviceGuard g(ctx->device);
    if (!ctx->use_graphs || ctx->profiling || n_iters < 2) {
        for (int it = 0; it < n_iters; ++it)
            if (int e = step(ctx)) return e;
        return SGTV_OK;
    }
    Context::Graph gr{};
    if (int e = context_graph(ctx, n_iters, &gr)) return e;
    HIP_TRY(hipGraphLaunch(gr.exec, ctx->stream));
    ctx->fcur = gr.fcur_after;
    ctx->vcur = gr.vcur_after;
    ctx->k += n_iters;
    return SGTV_OK;
}

int sgtv_prepare(sgtv_ctx ctx, int n_iters) {
    if (int e = check_ready(ctx)) return e;
    if (n_iters < 0) return fail(SGTV_EINVAL, "n_iters must be >= 0");
    if (!ctx->use_graphs || ctx->profiling || n_iters < 2) return SGTV_OK;
    DeviceGuard g(ctx->device);
    Context::Graph gr{};
    return context_graph(ctx, n_iters, &gr);
}

int sgtv_set_fused_update(sgtv_ctx ctx, int enable) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    DeviceGuard g(ctx->device);
    drop_graphs(ctx);
    ctx->fused = enable != 0;
    return SGTV_OK;
}

int sgtv_set_epilogues(sgtv_ctx ctx, int enable) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    DeviceGuard g(ctx->device);
    drop_graphs(ctx);
    ctx->epilogues = enable != 0;
    return SGTV_OK;
}

int sgtv_get_epilogues(sgtv_ctx ctx, int *enabled) {
    if (!ctx || !enabled) return fail(SGTV_EINVAL, "null argument");
    *enabled = ctx->epilogues ? 1 : 0;
    return SGTV_OK;
}

int sgtv_get_fused_update(sgtv_ctx ctx, int *active, int32_t *tile_x, int32_t *tile_y) {
    if (!ctx || !active) return fail(SGTV_EINVAL, "null argument");
    *active = ctx->sys ? (fused_ok(ctx) ? 1 : 0) : (ctx->fused ? 1 : 0);
    if (tile_x) *tile_x = ctx->sys ? ctx->sys->fused_tw : 0;
    if (tile_y) *tile_y = ctx->sys ? ctx->sys->fused_th : 0;
    return SGTV_OK;
}

int sgtv_set_graphs(sgtv_ctx ctx, int enable) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    DeviceGuard g(ctx->device);
    drop_graphs(ctx);
    ctx->use_graphs = enable != 0;
    return SGTV_OK;
}

namespace {

// Reduced report terms of the current state: h = [R(w.*Gf), ||w.*Gf - d||^2,
// ||(w.*G)^T (d - d_prev)||^2, ||w.*Gf||^2, ||d||^2, ||(w.*G)^T c||^2] (FP64).
int report_terms(sgtv_ctx ctx, double *dev_out, double h[6]) {
    const System &S = *ctx->sys;
    double *part = ctx->part.as<double>();
    int64_t n2 = 0;
    HIP_TRY(sgtv::launch_report(ctx->f[ctx->fcur].as<float>(), ctx->v[ctx->vcur].as<float>(),
                                ctx->a[ctx->vcur].as<float>(), ctx->v[ctx->vcur ^ 1].as<float>(),
                                ctx->a[ctx->vcur ^ 1].as<float>(), S.grid, S.weights(),
                                ctx->grouping, part, ctx->stream, &n2));
    HIP_TRY(sgtv::launch_reduce(part, n2, 6, dev_out, ctx->stream));
    if (h) {
        HIP_TRY(hipMemcpyAsync(h, dev_out, sizeof(double) * 6, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    return SGTV_OK;
}

}  // namespace

int sgtv_objective(sgtv_ctx ctx, sgtv_report *out) {
    if (int e = check_ready(ctx)) return e;
    if (!out) return fail(SGTV_EINVAL, "out is NULL");
    DeviceGuard g(ctx->device);
    const System &S = *ctx->sys;
    double *part = ctx->part.as<double>();
    double *red = ctx->red.as<double>();
    int64_t n1 = 0;
    const float *x = S.vt == SGTV_F32 ? ctx->f[ctx->fcur].as<float>() : ctx->fs.as<float>();
    if (S.format == SGTV_FORMAT_TILED) {
        HIP_TRY(sgtv::launch_tiled(S.fwd.map, S.vt, x, S.fpart.as<float>(), ctx->stream));
        HIP_TRY(sgtv::launch_ratio_combine(S.fpart.as<float>(), S.fwd.map.ns, S.I, ctx->y.as<float>(),
                                           ctx->r.as<float>(), ctx->ratio.as<float>(), part, true,
                                           ctx->stream, &n1));
    } else {
        HIP_TRY(sgtv::launch_forward_ratio(S.rows(), S.vt, x, ctx->y.as<float>(), ctx->r.as<float>(),
                                           ctx->ratio.as<float>(), part, true, ctx->stream, &n1));
    }
    HIP_TRY(sgtv::launch_reduce(part, n1, 1, red, ctx->stream));
    if (int e = report_terms(ctx, red + 1, nullptr)) return e;
    double h[4];
    HIP_TRY(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    out->data = h[0];
    out->tv = h[1];
    out->total = h[0] + ctx->beta * h[1];
    out->r_primal = std::sqrt(h[2]);
    out->r_dual = ctx->rho * std::sqrt(h[3]);
    out->iter = ctx->k;
    return SGTV_OK;
}

int sgtv_set_penalty(sgtv_ctx ctx, double rho) {
    if (int e = check_ready(ctx)) return e;
    if (!(std::isfinite(rho) && rho > 0.0)) return fail(SGTV_EINVAL, "rho must be finite and > 0");
    if (rho == ctx->rho) return SGTV_OK;
    DeviceGuard g(ctx->device);
    const float t = static_cast<float>(ctx->rho / rho);
    HIP_TRY(sgtv::launch_rescale_dual(ctx->v[ctx->vcur].as<float>(), ctx->a[ctx->vcur].as<float>(),
                                      ctx->sys->grid, ctx->grouping, t, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    drop_graphs(ctx);
    ctx->rho = rho;
    return SGTV_OK;
}

int sgtv_get_penalty(sgtv_ctx ctx, double *rho) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (!rho) return fail(SGTV_EINVAL, "rho is NULL");
    *rho = ctx->rho;
    return SGTV_OK;
}

int sgtv_iterate_adaptive(sgtv_ctx ctx, int64_t max_iters, const sgtv_adaptive *opt,
                          sgtv_check *checks, int32_t max_checks, int32_t *n_checks,
                          int64_t *iters_done, int *converged) {
    if (int e = check_ready(ctx)) return e;
    if (!opt) return fail(SGTV_EINVAL, "opt is NULL");
    if (max_iters < 0) return fail(SGTV_EINVAL, "max_iters must be >= 0");
    if (opt->check < 1) return fail(SGTV_EINVAL, "check must be >= 1");
    if (!(opt->eps_abs >= 0.0 && opt->eps_rel >= 0.0 && std::isfinite(opt->eps_abs) && std::isfinite(opt->eps_rel)))
        return fail(SGTV_EINVAL, "eps_abs and eps_rel must be finite and >= 0");
    if (!(opt->mu >= 1.0 && std::isfinite(opt->mu)) || !(opt->tau >= 1.0 && std::isfinite(opt->tau)))
        return fail(SGTV_EINVAL, "mu and tau must be finite and >= 1");
    if (max_checks < 0 || (max_checks > 0 && !checks)) return fail(SGTV_EINVAL, "checks is NULL");
    DeviceGuard g(ctx->device);
    const System &S = *ctx->sys;
    const double sq_p = std::sqrt(4.0 * static_cast<double>(S.J));
    const double sq_n = std::sqrt(static_cast<double>(S.J));
    int64_t k = 0;
    int32_t m = 0;
    int conv = 0;
    while (k < max_iters) {
        const int n = static_cast<int>(std::min<int64_t>(opt->check, max_iters - k));
        if (int e = sgtv_iterate(ctx, n)) return e;
        k += n;
        double h[6];
        if (int e = report_terms(ctx, ctx->red.as<double>() + 8, h)) return e;
        const double r = std::sqrt(h[1]), sd = ctx->rho * std::sqrt(h[2]);
        const double eps_pri = sq_p * opt->eps_abs + opt->eps_rel * std::max(std::sqrt(h[3]), std::sqrt(h[4]));
        const double eps_dual = sq_n * opt->eps_abs + opt->eps_rel * ctx->rho * std::sqrt(h[5]);
        const bool stop = r <= eps_pri && sd <= eps_dual;
        if (!stop) {
            double rho = ctx->rho;
            if (r > opt->mu * sd) rho *= opt->tau;
            else if (sd > opt->mu * r) rho /= opt->tau;
            if (int e = sgtv_set_penalty(ctx, rho)) return e;
        }
        if (m < max_checks) checks[m] = sgtv_check{k, r, sd, eps_pri, eps_dual, ctx->rho};
        ++m;
        if (stop) {
            conv = 1;
            break;
        }
    }
    if (n_checks) *n_checks = m;
    if (iters_done) *iters_done = k;
    if (converged) *converged = conv;
    return SGTV_OK;
}

int sgtv_get_image(sgtv_ctx ctx, float *x, int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    if (!x) return fail(SGTV_EINVAL, "x is NULL");
    DeviceGuard g(ctx->device);
    HIP_TRY(hipMemcpyAsync(x, ctx->f[ctx->fcur].p, sizeof(float) * ctx->sys->J, to_caller(mem_kind),
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SGTV_OK;
}

int sgtv_get_split(sgtv_ctx ctx, float *d, float *c, int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    DeviceGuard g(ctx->device);
    const System &S = *ctx->sys;
    DBuf td, tc;
    {
        ArenaScope sc(ws_section(ctx, &Workspace::temp), true);
        HIP_TRY(td.alloc(sizeof(float) * S.J * 4));
        HIP_TRY(tc.alloc(sizeof(float) * S.J * 4));
    }
    HIP_TRY(sgtv::launch_split_from_state(ctx->v[ctx->vcur].as<float>(), ctx->a[ctx->vcur].as<float>(),
                                          td.as<float>(), tc.as<float>(), S.grid, ctx->grouping,
                                          ctx->stream));
    if (d) HIP_TRY(hipMemcpyAsync(d, td.p, sizeof(float) * S.J * 4, to_caller(mem_kind), ctx->stream));
    if (c) HIP_TRY(hipMemcpyAsync(c, tc.p, sizeof(float) * S.J * 4, to_caller(mem_kind), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SGTV_OK;
}

int64_t sgtv_workspace_bytes(int64_t I, int64_t J, int64_t nnz, int storage_dtype) {
    if (I < 0 || J < 0 || nnz < 0) return -1;
    if (storage_dtype != SGTV_F32 && storage_dtype != SGTV_BF16 && storage_dtype != SGTV_F16) return -1;
    const int64_t vb = storage_dtype == SGTV_F32 ? 4 : 2;
    // one tiled copy with the automatic schedule: a list (rows of one wave x
    // one column block) of E entries takes max(E / 64 + 1, longest row run)
    // groups of 64, the run estimated for rows with lam entries per block
    auto copy_bytes = [&](int64_t n_rows, int64_t n_cols, int64_t *slabs) -> double {
        const TileParams t = choose_tiles(n_rows, n_cols, 16, 0, 0, 0);
        *slabs = t.ns;
        if (n_rows == 0 || n_cols == 0) return 0.0;
        const double n_rb = std::ceil(static_cast<double>(n_rows) / (16.0 * t.rw));
        const double ncb = std::ceil(static_cast<double>(n_cols) / t.cb);
        const double lists = n_rb * ncb * 16.0;
        const double lam = static_cast<double>(nnz) / n_rows * std::min<double>(t.cb, n_cols) / n_cols;
        const double e = static_cast<double>(nnz) / lists;
        const double groups = std::max(std::ceil(e / 64.0) + 1.0, std::ceil(lam + 2.5 * std::sqrt(lam) + 1.0));
        const double stored = std::min(lists * 64.0 * groups, 64.0 * static_cast<double>(nnz) + 256.0);
        const bool i24 = sgtv::idx24_fits(t.rw, t.cb);
        const double idx_bytes = i24 ? 3.0 : 4.0;
        // 24-bit lists also keep the row order of every tile (2 bytes per row and slab)
        const double order = i24 ? 2.0 * n_rb * 16.0 * t.rw * t.ns : 0.0;
        return stored * (idx_bytes + vb) + lists * 8.0 + order;
    };
    int64_t ns_f = 1, ns_b = 1;
    const double matrix = copy_bytes(I, J, &ns_f) + copy_bytes(J, I, &ns_b);
    const int64_t vectors = 4 * (3 * J + 2 * 4 * J + 2 * J + 2 * J)   // f x2, fs, v x2, a x2, sens, H
                            + 4 * 3 * I                                   // y, r, ratio
                            + 4 * (ns_f * I + ns_b * J)                   // partial sums
                            + (storage_dtype == SGTV_F32 ? 0 : 4 * J);    // column scales
    return static_cast<int64_t>(matrix) + vectors + (1 << 20);
}

int sgtv_device_bytes(sgtv_ctx ctx, int64_t *bytes) {
    if (!ctx || !bytes) return fail(SGTV_EINVAL, "null argument");
    int64_t b = 0;
    auto add = [&](const DBuf *d) {
        if (!d->borrowed) b += static_cast<int64_t>(d->bytes);
    };
    for (const DBuf *d : {&ctx->y, &ctx->r, &ctx->ratio, &ctx->f[0], &ctx->f[1], &ctx->v[0], &ctx->v[1],
                          &ctx->a[0], &ctx->a[1], &ctx->fs, &ctx->part, &ctx->red})
        add(d);
    if (ctx->sys) {
        const System &S = *ctx->sys;
        for (const DBuf *d : {&S.rs_ptr, &S.rs_idx, &S.rs_val, &S.cs_ptr, &S.cs_idx, &S.cs_val, &S.colscale,
                              &S.sens, &S.H, &S.htab, &S.wbuf, &S.fpart, &S.bpart, &S.fwd.pk, &S.fwd.val,
                              &S.fwd.goff, &S.fwd.poff, &S.fwd.slot, &S.back.pk, &S.back.val, &S.back.goff,
                              &S.back.poff, &S.back.slot, &S.fcount, &S.bcount})
            add(d);
    }
    *bytes = b;
    return SGTV_OK;
}

int sgtv_state_sizes(sgtv_ctx ctx, int64_t *n_image, int64_t *n_split, int64_t *n_gr) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (!ctx->sys) return fail(SGTV_ESTATE, "no system set");
    if (n_image) *n_image = ctx->sys->J;
    if (n_split) *n_split = ctx->sys->J * 4;
    if (n_gr) *n_gr = n_groups(ctx);
    return SGTV_OK;
}

int sgtv_get_state(sgtv_ctx ctx, float *f, float *v, float *a, int64_t *k, int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    DeviceGuard g(ctx->device);
    const System &S = *ctx->sys;
    if (f) HIP_TRY(hipMemcpyAsync(f, ctx->f[ctx->fcur].p, sizeof(float) * S.J, to_caller(mem_kind), ctx->stream));
    if (v) HIP_TRY(hipMemcpyAsync(v, ctx->v[ctx->vcur].p, sizeof(float) * S.J * 4, to_caller(mem_kind), ctx->stream));
    if (a) HIP_TRY(hipMemcpyAsync(a, ctx->a[ctx->vcur].p, sizeof(float) * n_groups(ctx), to_caller(mem_kind), ctx->stream));
    if (k) *k = ctx->k;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SGTV_OK;
}

static bool finite_any(float x) { return std::isfinite(x); }
static bool unit_interval(float x) { return std::isfinite(x) && x >= 0.0f && x <= 1.0f; }

int sgtv_set_state(sgtv_ctx ctx, const float *f, const float *v, const float *a, int64_t k,
                   int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    if (!f || !v || !a) return fail(SGTV_EINVAL, "f, v and a are required");
    if (k < 0) return fail(SGTV_EINVAL, "k must be >= 0");
    DeviceGuard g(ctx->device);
    try {
        const System &S = *ctx->sys;
        DBuf sf, sv, sa;
        ArenaScope sc(ws_section(ctx, &Workspace::temp), true);
        if (int e = stage_floats(sf, f, S.J, mem_kind, ctx->stream, finite_nonneg, "f")) return e;
        if (int e = stage_floats(sv, v, S.J * 4, mem_kind, ctx->stream, finite_any, "v")) return e;
        if (int e = stage_floats(sa, a, n_groups(ctx), mem_kind, ctx->stream, unit_interval, "a")) return e;
        drop_graphs(ctx);
        ctx->fcur = 0;
        ctx->vcur = 0;
        HIP_TRY(hipMemcpyAsync(ctx->f[0].p, sf.p, sizeof(float) * S.J, hipMemcpyDeviceToDevice, ctx->stream));
        for (int b = 0; b < 2; ++b) {
            HIP_TRY(hipMemcpyAsync(ctx->v[b].p, sv.p, sizeof(float) * S.J * 4, hipMemcpyDeviceToDevice, ctx->stream));
            HIP_TRY(hipMemcpyAsync(ctx->a[b].p, sa.p, sizeof(float) * n_groups(ctx), hipMemcpyDeviceToDevice, ctx->stream));
        }
        ctx->k = k;
        if (int e = refresh_scaled(ctx)) return e;
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

int sgtv_backprojection(sgtv_ctx ctx, float *x, int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    if (!x) return fail(SGTV_EINVAL, "x is NULL");
    DeviceGuard g(ctx->device);
    const System &S = *ctx->sys;
    DBuf e, out;
    {
        ArenaScope sc(ws_section(ctx, &Workspace::temp), true);
        HIP_TRY(e.alloc(sizeof(float) * S.J));
        HIP_TRY(out.alloc(sizeof(float) * S.J));
    }
    if (int st = back_project(S, ctx->y.as<float>(), e.as<float>(), ctx->stream)) return st;
    HIP_TRY(sgtv::launch_div_safe(e.as<float>(), S.sens.as<float>(), out.as<float>(), S.J, ctx->stream));
    HIP_TRY(hipMemcpyAsync(x, out.p, sizeof(float) * S.J, to_caller(mem_kind), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SGTV_OK;
}

int sgtv_backprojection_noalloc(sgtv_ctx ctx, float *x, int mem_kind) {
    if (int e = check_ready(ctx)) return e;
    if (int e = check_mem_kind(mem_kind)) return e;
    if (!x) return fail(SGTV_EINVAL, "x is NULL");
    const System &S = *ctx->sys;
    if (2 * S.J > kScratchFloats)
        return fail(SGTV_ESHAPE, "sgtv_backprojection_noalloc takes at most " + std::to_string(kScratchFloats / 2) +
                                     " hyper-voxels (J = " + std::to_string(S.J) + ")");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SGTV_EDEVICE, "cannot select device");
    float *buf = nullptr;
    HIP_TRY(scratch_address(ctx->device, &buf));
    // A^T y in the first J floats of the buffer, the quotient in the next J
    float *e = buf, *q = buf + S.J;
    if (int st = back_project(S, ctx->y.as<float>(), e, ctx->stream)) return st;
    HIP_TRY(sgtv::launch_div_safe(e, S.sens.as<float>(), q, S.J, ctx->stream));
    HIP_TRY(hipMemcpyAsync(x, q, sizeof(float) * S.J, to_caller(mem_kind), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SGTV_OK;
}

int sgtv_set_schedule(sgtv_ctx ctx, const sgtv_schedule *s) {
    if (!ctx || !s) return fail(SGTV_EINVAL, "null argument");
    if (s->format != SGTV_FORMAT_TILED && s->format != SGTV_FORMAT_SELL) return fail(SGTV_EINVAL, "unknown format");
    if (s->waves < 0 || s->waves > 16) return fail(SGTV_EINVAL, "waves must be in [1, 16] (0: automatic)");
    if (s->variant < 0 || s->variant > 3) return fail(SGTV_EINVAL, "variant must be in [1, 3] (0: automatic)");
    const int32_t rws[2] = {s->fwd_rows_per_wave, s->back_rows_per_wave};
    const int32_t cbs[2] = {s->fwd_block_cols, s->back_block_cols};
    const int32_t nss[2] = {s->fwd_slabs, s->back_slabs};
    for (int i = 0; i < 2; ++i) {
        if (rws[i] < 0 || rws[i] > 32767) return fail(SGTV_EINVAL, "rows_per_wave must be in [1, 32767]");
        if (cbs[i] < 0 || cbs[i] > 65536 || (cbs[i] % 4) != 0) return fail(SGTV_EINVAL, "block_cols must be a multiple of 4 in [4, 65536]");
        if (nss[i] < 0 || nss[i] > sgtv::kMaxSlabs) return fail(SGTV_EINVAL, "slabs must be in [1, 16]");
    }
    ctx->want = *s;
    return SGTV_OK;
}

int sgtv_get_schedule(sgtv_ctx ctx, sgtv_schedule *s) {
    if (!ctx || !s) return fail(SGTV_EINVAL, "null argument");
    *s = ctx->sys ? ctx->sys->sched : ctx->want;
    return SGTV_OK;
}

int sgtv_set_profiling(sgtv_ctx ctx, int enable) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    ctx->profiling = enable != 0;
    return SGTV_OK;
}

int sgtv_kernel_times(sgtv_ctx ctx, double *ms, int64_t *counts) {
    if (!ctx) return fail(SGTV_EINVAL, "null context");
    if (!ms || !counts) return fail(SGTV_EINVAL, "ms and counts (5 entries each) are required");
    DeviceGuard g(ctx->device);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    int status = SGTV_OK;
    for (auto &t : ctx->timed) {
        float el = 0.0f;
        hipError_t e = hipEventElapsedTime(&el, t.beg, t.end);
        if (e != hipSuccess && status == SGTV_OK) status = hip_fail(e, "hipEventElapsedTime");
        if (e == hipSuccess && t.cls >= 0 && t.cls < 5) {
            ms[t.cls] += el;
            counts[t.cls] += 1;
        }
        (void)hipEventDestroy(t.beg);
        (void)hipEventDestroy(t.end);
    }
    ctx->timed.clear();
    return status;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct sgtv_batch_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;                    // add_scan may be called from several threads
    std::vector<sgtv_ctx_s *> scans;
    bool dirty = true;
    // device tables
    DBuf tiles_f, tiles_b, maps_f, maps_b, xs_f[2], xs_b, parts_f, parts_b, scandev;
    DBuf rblocks, vblocks, sblocks;
    int64_t n_tiles_f = 0, n_tiles_b = 0, n_rblocks = 0, n_vblocks = 0, n_sblocks = 0;
    size_t lds_f = 0, lds_b = 0;
    int waves = 16, variant = 1;
    int storage = SGTV_F32;           // value type of every scan's matrix (one product launch per type)
    int fcur = 0, vcur = 0;
    hipStream_t cap = nullptr;
    std::vector<sgtv_ctx_s::Graph> graphs;
    // persistent launch: arrival counter and error flag of its grid barriers
    int launch = SGTV_BATCH_GRAPH;
    DBuf bar, pdev, ticks;            // barrier and queue counters; the kernel's table; phase clocks
    sgtv::PersistentDev pdev_host{};
    int persistent_grid = 0;
    int64_t persistent_iters = 0;     // iterations behind the phase clocks
    ~sgtv_batch_s() {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
        if (cap) (void)hipStreamDestroy(cap);
        for (auto *c : scans) {
            drop_graphs(c);
            if (c->cap) (void)hipStreamDestroy(c->cap);
            delete c;
        }
    }
};

namespace {

template <class T>
hipError_t upload_vec(DBuf &d, const std::vector<T> &h) { return upload(d, h); }

int batch_tables(sgtv_batch_s *b) {
    const size_t n = b->scans.size();
    // scans by decreasing nonzeros: large tiles first, small ones fill the tail
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        return b->scans[x]->sys->nnz > b->scans[y]->sys->nnz;
    });
    std::vector<sgtv::BatchTile> tf, tb;
    std::vector<sgtv::TileMap> mf(n), mb(n);
    std::vector<const float *> xf0(n), xf1(n), xb(n);
    std::vector<float *> pf(n), pb(n);
    std::vector<sgtv::ScanDev> sd(n);
    std::vector<sgtv::BatchBlock> rbl, vbl, sbl;
    b->lds_f = b->lds_b = 0;
    for (size_t i = 0; i < n; ++i) {
        sgtv_ctx_s *c = b->scans[i];
        const System &S = *c->sys;
        mf[i] = S.fwd.map;
        mb[i] = S.back.map;
        // the forward product reads the image, or its scaled copy for 16-bit values
        xf0[i] = S.vt == SGTV_F32 ? c->f[0].as<float>() : c->fs.as<float>();
        xf1[i] = S.vt == SGTV_F32 ? c->f[1].as<float>() : c->fs.as<float>();
        xb[i] = c->ratio.as<float>();
        pf[i] = S.fpart.as<float>();
        pb[i] = S.bpart.as<float>();
        b->lds_f = std::max(b->lds_f, S.fwd.map.lds_bytes());
        b->lds_b = std::max(b->lds_b, S.back.map.lds_bytes());
        sgtv::ScanDev &d = sd[i];
        d.y = c->y.as<float>();
        d.r = c->r.as<float>();
        d.ratio = c->ratio.as<float>();
        d.fpart = S.fpart.as<float>();
        d.bpart = S.bpart.as<float>();
        for (int k = 0; k < 2; ++k) {
            d.f[k] = c->f[k].as<float>();
            d.v[k] = c->v[k].as<float>();
            d.a[k] = c->a[k].as<float>();
        }
        d.sens = S.sens.as<float>();
        d.H = S.H.as<float>();
        d.htab = S.htab.as<float>();
        d.scale = S.vt == SGTV_F32 ? nullptr : S.colscale.as<float>();
        d.fs = S.vt == SGTV_F32 ? nullptr : c->fs.as<float>();
        d.grid = S.grid;
        d.wts = S.weights();
        d.grouping = c->grouping;
        d.I = S.I;
        d.ns_f = S.fwd.map.ns;
        d.ns_b = S.back.map.ns;
        int sl = 0;
        while ((1 << sl) < S.Q && sl < 6) ++sl;
        d.seg_log2 = sl;
        d.lam = static_cast<float>(c->rho);
        d.thr = static_cast<float>(c->beta / c->rho);
    }
    for (size_t oi = 0; oi < n; ++oi) {
        const int32_t i = static_cast<int32_t>(order[oi]);
        const System &S = *b->scans[i]->sys;
        // tiles of one scan start at a multiple of 8 so each slab keeps its XCDs
        auto add_tiles = [&](std::vector<sgtv::BatchTile> &t, const sgtv::TileMap &M) {
            const int64_t nt = M.n_rb * M.ns;
            for (int64_t k = 0; k < nt; ++k) t.push_back({i, static_cast<int32_t>(k)});
            while (t.size() % 8) t.push_back({i, -1});
        };
        add_tiles(tf, S.fwd.map);
        add_tiles(tb, S.back.map);
        for (int64_t st = 0; st < S.I; st += sgtv::kBlock) rbl.push_back({i, 0, st});
        for (int64_t st = 0; st < S.J; st += sgtv::kBlock) vbl.push_back({i, 0, st});
        const int64_t segs = sgtv::kBlock >> sd[i].seg_log2;
        for (int64_t st = 0; st < S.S; st += segs) sbl.push_back({i, 0, st});
    }
    HIP_TRY(upload_vec(b->tiles_f, tf));
    HIP_TRY(upload_vec(b->tiles_b, tb));
    HIP_TRY(upload_vec(b->maps_f, mf));
    HIP_TRY(upload_vec(b->maps_b, mb));
    HIP_TRY(upload_vec(b->xs_f[0], xf0));
    HIP_TRY(upload_vec(b->xs_f[1], xf1));
    HIP_TRY(upload_vec(b->xs_b, xb));
    HIP_TRY(upload_vec(b->parts_f, pf));
    HIP_TRY(upload_vec(b->parts_b, pb));
    HIP_TRY(upload_vec(b->scandev, sd));
    HIP_TRY(upload_vec(b->rblocks, rbl));
    HIP_TRY(upload_vec(b->vblocks, vbl));
    HIP_TRY(upload_vec(b->sblocks, sbl));
    b->n_tiles_f = static_cast<int64_t>(tf.size());
    b->n_tiles_b = static_cast<int64_t>(tb.size());
    b->n_rblocks = static_cast<int64_t>(rbl.size());
    b->n_vblocks = static_cast<int64_t>(vbl.size());
    b->n_sblocks = static_cast<int64_t>(sbl.size());
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
    b->dirty = false;
    return SGTV_OK;
}

int batch_step(sgtv_batch_s *b) {
    hipStream_t st = b->stream;
    HIP_TRY(sgtv::launch_tiled_batch(b->tiles_f.as<sgtv::BatchTile>(), b->n_tiles_f,
                                     b->maps_f.as<sgtv::TileMap>(), b->xs_f[b->fcur].as<const float *>(),
                                     b->parts_f.as<float *>(), b->waves, b->lds_f, b->variant, b->storage, st));
    HIP_TRY(sgtv::launch_ratio_batch(b->rblocks.as<sgtv::BatchBlock>(), b->n_rblocks,
                                     b->scandev.as<sgtv::ScanDev>(), st));
    HIP_TRY(sgtv::launch_tiled_batch(b->tiles_b.as<sgtv::BatchTile>(), b->n_tiles_b,
                                     b->maps_b.as<sgtv::TileMap>(), b->xs_b.as<const float *>(),
                                     b->parts_b.as<float *>(), b->waves, b->lds_b, b->variant, b->storage, st));
    HIP_TRY(sgtv::launch_voxel_batch(b->vblocks.as<sgtv::BatchBlock>(), b->n_vblocks,
                                     b->scandev.as<sgtv::ScanDev>(), b->fcur, b->vcur, st));
    b->fcur ^= 1;
    HIP_TRY(sgtv::launch_split_batch(b->sblocks.as<sgtv::BatchBlock>(), b->n_sblocks,
                                     b->scandev.as<sgtv::ScanDev>(), b->fcur, b->vcur, st));
    b->vcur ^= 1;
    return SGTV_OK;
}

void batch_sync_scans(sgtv_batch_s *b, int n_iters) {
    for (auto *c : b->scans) {
        c->fcur = b->fcur;
        c->vcur = b->vcur;
        c->k += n_iters;
    }
}

// Iterations per cooperative launch: the barrier counter (4 arrivals of every
// workgroup per iteration) stays far below 2^32.
constexpr int kPersistentChunk = 100000;
// Longest wait at one grid barrier before the launch is abandoned.
constexpr double kBarrierLimitSeconds = 2.0;

// n_iters iterations of every scan in cooperative launches of the persistent
// kernel; waits for them and reports a barrier that timed out.
int batch_persistent(sgtv_batch_s *b, int n_iters) {
    if (b->storage != SGTV_F32) return fail(SGTV_EINVAL, "the persistent launch runs batches of FP32 values only");
    if (b->dirty)
        if (int e = batch_tables(b)) return e;
    if (b->waves % 4 != 0)
        return fail(SGTV_EINVAL, "the persistent launch needs a multiple of 4 waves per workgroup");
    if (!b->bar.p) HIP_TRY(b->bar.alloc(sizeof(uint32_t) * sgtv::kBarWords));
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
    if (khz <= 0) return fail(SGTV_EDEVICE, "no wall-clock rate for the grid barriers");
    const uint64_t limit = static_cast<uint64_t>(kBarrierLimitSeconds * 1000.0 * khz);
    if (!b->pdev.p) HIP_TRY(b->pdev.alloc(sizeof(sgtv::PersistentDev)));
    if (!b->ticks.p) {
        HIP_TRY(b->ticks.alloc(sizeof(uint64_t) * sgtv::kPhaseSlots));
        HIP_TRY(hipMemsetAsync(b->ticks.p, 0, sizeof(uint64_t) * sgtv::kPhaseSlots, b->stream));
    }
    {
        sgtv::PersistentDev &D = b->pdev_host;
        D.tiles_f = b->tiles_f.as<sgtv::BatchTile>();
        D.tiles_b = b->tiles_b.as<sgtv::BatchTile>();
        D.maps_f = b->maps_f.as<sgtv::TileMap>();
        D.maps_b = b->maps_b.as<sgtv::TileMap>();
        D.xs_f0 = b->xs_f[0].as<const float *>();
        D.xs_f1 = b->xs_f[1].as<const float *>();
        D.xs_b = b->xs_b.as<const float *>();
        D.parts_f = b->parts_f.as<float *>();
        D.parts_b = b->parts_b.as<float *>();
        D.scans = b->scandev.as<sgtv::ScanDev>();
        D.rblocks = b->rblocks.as<sgtv::BatchBlock>();
        D.vblocks = b->vblocks.as<sgtv::BatchBlock>();
        D.sblocks = b->sblocks.as<sgtv::BatchBlock>();
        D.bar = b->bar.as<uint32_t>();
        D.limit = limit;
        D.ticks = b->ticks.as<uint64_t>();
        HIP_TRY(hipMemcpyAsync(b->pdev.p, &D, sizeof(D), hipMemcpyHostToDevice, b->stream));
    }
    for (int done = 0; done < n_iters;) {
        const int n = std::min(n_iters - done, kPersistentChunk);
        HIP_TRY(hipMemsetAsync(b->bar.p, 0, sizeof(uint32_t) * sgtv::kBarWords, b->stream));
        const sgtv::PersistentPlan plan{b->n_tiles_f, b->n_tiles_b, b->n_rblocks, b->n_vblocks, b->n_sblocks,
                                        n, b->fcur, b->vcur, b->waves / 4};
        const size_t lds = std::max(b->lds_f, b->lds_b);
        const int threads = b->waves * sgtv::kWave;
        const char *what = "";
        if (hipError_t e = sgtv::persistent_grid(b->variant, threads, lds, &b->persistent_grid, &what))
            return hip_fail(e, (std::string("persistent launch: ") + what).c_str());
        if (hipError_t e = sgtv::launch_admm_persistent(b->pdev.as<sgtv::PersistentDev>(), plan, lds, threads,
                                                        b->variant, b->persistent_grid, b->stream))
            return hip_fail(e, ("persistent launch: hipLaunchCooperativeKernel (grid " +
                                std::to_string(b->persistent_grid) + " x " + std::to_string(threads) +
                                " threads, " + std::to_string(lds) + " bytes of LDS)").c_str());
        int err = 0;
        HIP_TRY(hipMemcpyAsync(&err, b->bar.as<int>() + sgtv::kBarErr, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        if (err)
            return fail(SGTV_EDEVICE, "persistent launch: a grid barrier waited longer than its limit and the "
                                      "launch was abandoned; the batch state is undefined");
        if (n & 1) {
            b->fcur ^= 1;
            b->vcur ^= 1;
        }
        batch_sync_scans(b, n);
        b->persistent_iters += n;
        done += n;
    }
    return SGTV_OK;
}

int batch_join(sgtv_batch_s *b, std::unique_ptr<sgtv_ctx_s> own, const float *y, const float *r, double beta,
               double rho, int grouping, int mem_kind, int32_t *index);

}  // namespace

extern "C" {

int sgtv_batch_create(sgtv_batch *out, int device, void *hip_stream) {
    if (!out) return fail(SGTV_EINVAL, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(SGTV_EINVAL, "device index out of range");
    try {
        auto b = new sgtv_batch_s();
        b->device = device;
        b->stream = static_cast<hipStream_t>(hip_stream);
        *out = b;
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

void sgtv_batch_destroy(sgtv_batch b) {
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    delete b;
}

int sgtv_batch_add_scan(sgtv_batch b, int64_t I, int32_t ny, int32_t nx, int32_t Q,
                        const int64_t *row_ptr, const int32_t *col_idx, const float *val,
                        int64_t nnz, const float *w, int64_t w_len, const float *y, const float *r,
                        double beta, double rho, int grouping, const sgtv_schedule *schedule,
                        int mem_kind, int32_t *index) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    {
        std::lock_guard<std::mutex> lock(b->mu);
        if (b->scans.size() >= (size_t(1) << 30)) return fail(SGTV_ESHAPE, "too many scans");
        // keep the batch in lockstep: a new scan may only join before the first iteration
        if (!b->scans.empty() && b->scans.front()->k != 0)
            return fail(SGTV_ESTATE, "scans can only be added before the batch iterates");
    }
    sgtv_ctx c = nullptr;
    if (int e = sgtv_create(&c, b->device, b->stream)) return e;
    std::unique_ptr<sgtv_ctx_s> own(c);
    sgtv_schedule sch{};
    if (schedule) sch = *schedule;
    sch.format = SGTV_FORMAT_TILED;
    if (int e = sgtv_set_schedule(c, &sch)) return e;
    if (int e = sgtv_set_system(c, I, ny, nx, Q, row_ptr, col_idx, val, nnz, b->storage, w, w_len, mem_kind))
        return e;
    return batch_join(b, std::move(own), y, r, beta, rho, grouping, mem_kind, index);
}

int sgtv_batch_add_system_file(sgtv_batch b, const char *path, const float *y, const float *r, double beta,
                               double rho, int grouping, int mem_kind, int32_t *index) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    sgtv_ctx c = nullptr;
    if (int e = sgtv_create(&c, b->device, b->stream)) return e;
    std::unique_ptr<sgtv_ctx_s> own(c);
    if (int e = sgtv_load_system(c, path)) return e;
    if (c->sys->format != SGTV_FORMAT_TILED || c->sys->vt != b->storage)
        return fail(SGTV_EINVAL, "scans of a batch need a tiled system with the batch's value type");
    return batch_join(b, std::move(own), y, r, beta, rho, grouping, mem_kind, index);
}

int sgtv_batch_save_scan(sgtv_batch b, int32_t scan, const char *path) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    sgtv_ctx_s *c = nullptr;
    {
        std::lock_guard<std::mutex> lock(b->mu);
        if (scan < 0 || static_cast<size_t>(scan) >= b->scans.size()) return fail(SGTV_EINVAL, "scan out of range");
        c = b->scans[scan];
    }
    return sgtv_save_system(c, path);
}

}  // extern "C"

namespace {

// Joins a scan whose system is set to the batch: grouping and data, then the
// check that it shares waves and variant with the scans already there.
int batch_join(sgtv_batch_s *b, std::unique_ptr<sgtv_ctx_s> own, const float *y, const float *r, double beta,
               double rho, int grouping, int mem_kind, int32_t *index) {
    sgtv_ctx_s *c = own.get();
    if (int e = sgtv_set_grouping(c, grouping)) return e;
    if (int e = sgtv_set_data(c, y, r, beta, rho, 1, mem_kind)) return e;
    std::lock_guard<std::mutex> lock(b->mu);
    if (!b->scans.empty() && b->scans.front()->k != 0)
        return fail(SGTV_ESTATE, "scans can only be added before the batch iterates");
    const sgtv_schedule &got = c->sys->sched;
    if (!b->scans.empty()) {
        const sgtv_schedule &first = b->scans.front()->sys->sched;
        if (got.waves != first.waves || got.variant != first.variant)
            return fail(SGTV_EINVAL, "scans of one batch must share waves and variant");
    } else {
        b->waves = got.waves;
        b->variant = got.variant - 1;
    }
    b->scans.push_back(own.release());
    b->dirty = true;
    if (index) *index = static_cast<int32_t>(b->scans.size() - 1);
    return SGTV_OK;
}

}  // namespace

extern "C" {

int sgtv_batch_size(sgtv_batch b, int32_t *n_scans) {
    if (!b || !n_scans) return fail(SGTV_EINVAL, "null argument");
    *n_scans = static_cast<int32_t>(b->scans.size());
    return SGTV_OK;
}

namespace {

// The graph of n_iters batched iterations from the current buffer parity:
// found in the cache or captured (not run) and instantiated.
int batch_graph(sgtv_batch b, int n_iters, sgtv_ctx_s::Graph *out) {
    if (b->dirty)
        if (int e = batch_tables(b)) return e;
    for (auto &gr : b->graphs)
        if (gr.n == n_iters && gr.fcur == b->fcur && gr.vcur == b->vcur) {
            *out = gr;
            return SGTV_OK;
        }
    if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    const int f0 = b->fcur, v0 = b->vcur;
    hipStream_t user = b->stream;
    b->stream = b->cap;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
    int status = e == hipSuccess ? SGTV_OK : hip_fail(e, "hipStreamBeginCapture");
    for (int it = 0; it < n_iters && status == SGTV_OK && e == hipSuccess; ++it) status = batch_step(b);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) {
        hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
        if (status == SGTV_OK && e2 != hipSuccess) status = hip_fail(e2, "hipStreamEndCapture");
    }
    b->stream = user;
    sgtv_ctx_s::Graph gr{n_iters, f0, v0, b->fcur, b->vcur, nullptr};
    b->fcur = f0;
    b->vcur = v0;
    if (status == SGTV_OK) {
        hipError_t e3 = hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0);
        if (e3 != hipSuccess) status = hip_fail(e3, "hipGraphInstantiate");
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (status != SGTV_OK) return status;
    if (b->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(b->graphs.front().exec);
        b->graphs.erase(b->graphs.begin());
    }
    b->graphs.push_back(gr);
    *out = gr;
    return SGTV_OK;
}

}  // namespace

int sgtv_batch_iterate(sgtv_batch b, int n_iters) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    if (n_iters < 0) return fail(SGTV_EINVAL, "n_iters must be >= 0");
    if (b->scans.empty() || n_iters == 0) return SGTV_OK;
    DeviceGuard g(b->device);
    if (b->launch == SGTV_BATCH_PERSISTENT) return batch_persistent(b, n_iters);
    sgtv_ctx_s::Graph gr{};
    if (int e = batch_graph(b, n_iters, &gr)) return e;
    HIP_TRY(hipGraphLaunch(gr.exec, b->stream));
    b->fcur = gr.fcur_after;
    b->vcur = gr.vcur_after;
    batch_sync_scans(b, n_iters);
    return SGTV_OK;
}

int sgtv_batch_prepare(sgtv_batch b, int n_iters, int sequential) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    if (n_iters < 0) return fail(SGTV_EINVAL, "n_iters must be >= 0");
    if (sequential != 0 && sequential != 1) return fail(SGTV_EINVAL, "sequential must be 0 or 1");
    if (sequential) {
        for (auto *c : b->scans)
            if (int e = sgtv_prepare(c, n_iters)) return e;
        return SGTV_OK;
    }
    if (b->scans.empty() || n_iters == 0) return SGTV_OK;
    DeviceGuard g(b->device);
    if (b->launch == SGTV_BATCH_PERSISTENT) return b->dirty ? batch_tables(b) : SGTV_OK;
    sgtv_ctx_s::Graph gr{};
    return batch_graph(b, n_iters, &gr);
}

int sgtv_batch_iterate_sequential(sgtv_batch b, int n_iters) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    if (n_iters < 0) return fail(SGTV_EINVAL, "n_iters must be >= 0");
    for (auto *c : b->scans)
        if (int e = sgtv_iterate(c, n_iters)) return e;
    if (!b->scans.empty()) {
        b->fcur = b->scans.front()->fcur;
        b->vcur = b->scans.front()->vcur;
    }
    return SGTV_OK;
}

int sgtv_batch_set_storage(sgtv_batch b, int storage_dtype) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    if (storage_dtype != SGTV_F32 && storage_dtype != SGTV_BF16 && storage_dtype != SGTV_F16)
        return fail(SGTV_EINVAL, "unknown storage dtype");
    std::lock_guard<std::mutex> lock(b->mu);
    if (!b->scans.empty()) return fail(SGTV_ESTATE, "the value type is set before the first scan is added");
    b->storage = storage_dtype;
    return SGTV_OK;
}

int sgtv_batch_set_launch(sgtv_batch b, int mode) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    if (mode != SGTV_BATCH_GRAPH && mode != SGTV_BATCH_PERSISTENT)
        return fail(SGTV_EINVAL, "launch mode must be SGTV_BATCH_GRAPH or SGTV_BATCH_PERSISTENT");
    b->launch = mode;
    return SGTV_OK;
}

int sgtv_batch_get_launch(sgtv_batch b, int *mode, int32_t *grid) {
    if (!b || !mode) return fail(SGTV_EINVAL, "null argument");
    *mode = b->launch;
    if (grid) *grid = b->persistent_grid;
    return SGTV_OK;
}

int sgtv_batch_phase_times(sgtv_batch b, double *ms, int64_t *iters) {
    if (!b || !ms || !iters) return fail(SGTV_EINVAL, "null argument");
    for (int k = 0; k < sgtv::kPhaseSlots; ++k) ms[k] = 0.0;
    *iters = b->persistent_iters;
    if (!b->ticks.p) return SGTV_OK;
    DeviceGuard g(b->device);
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
    uint64_t t[sgtv::kPhaseSlots] = {};
    HIP_TRY(hipMemcpyAsync(t, b->ticks.p, sizeof(t), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipMemsetAsync(b->ticks.p, 0, sizeof(t), b->stream));
    for (int k = 0; k < sgtv::kPhaseSlots; ++k) ms[k] = khz > 0 ? static_cast<double>(t[k]) / khz : 0.0;
    b->persistent_iters = 0;
    return SGTV_OK;
}

int sgtv_batch_objective(sgtv_batch b, int32_t scan, sgtv_report *out) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    if (scan < 0 || static_cast<size_t>(scan) >= b->scans.size()) return fail(SGTV_EINVAL, "scan index out of range");
    return sgtv_objective(b->scans[scan], out);
}

int sgtv_batch_get_image(sgtv_batch b, int32_t scan, float *x, int mem_kind) {
    if (!b) return fail(SGTV_EINVAL, "null batch");
    if (scan < 0 || static_cast<size_t>(scan) >= b->scans.size()) return fail(SGTV_EINVAL, "scan index out of range");
    return sgtv_get_image(b->scans[scan], x, mem_kind);
}

}  // extern "C"

// ------------------------------------------------------------------ warm-start network

struct wsnet_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int L = 0, H = 0, W = 0, C = 0, max_batch = 0;
    int64_t n_param = 0, per_layer = 0, img = 0;   // img = H * W * C
    DBuf params, grad, m, v;                        // FP32
    DBuf wf, wb;                                    // bf16 weights, L blocks of C*9*C
    DBuf acts;                                      // bf16 inputs of every layer
    DBuf z_last, out, xin, tgt;                     // FP32
    DBuf dz[2];                                     // bf16 gradients w.r.t. pre-activations
    DBuf wpart, lpart, lred;
    DBuf lsum;                                      // FP64 sum of the training steps' losses and their count
    DBuf xt, dt;                                    // weight gradient: X of every layer in three
                                                    // shifted channel-major copies; dZ channel-major
    DBuf ipart, isum;                               // per-image FP64 sums (start images)
    int64_t step = 0;
    bool have_grad = false, have_params = false;
};

namespace {

constexpr int kLossBlocks = 4096;   // loss-gradient blocks (FP64 partial sums of the squared error)
constexpr int kImageBlocks = 64;    // partial sums per image (start images)

__bf16 *bf(const DBuf &b, int64_t off = 0) { return b.as<__bf16>() + off; }

int net_weights(wsnet_s *n) {
    for (int l = 0; l < n->L; ++l)
        HIP_TRY(sgtv::wsn::weights_bf16(n->params.as<float>() + l * n->per_layer,
                                        bf(n->wf, l * n->C * 9 * n->C), bf(n->wb, l * n->C * 9 * n->C),
                                        n->stream));
    return SGTV_OK;
}

int net_stage(wsnet_s *n, DBuf &dst, const float *src, int64_t count, int mk) {
    HIP_TRY(hipMemcpyAsync(dst.p, src, sizeof(float) * count,
                           mk == SGTV_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, n->stream));
    return SGTV_OK;
}

// the layers, from the bf16 input already in the first activation buffer;
// training: the hidden layers also write their outputs' shifted channel-major
// copies for the weight gradients
int net_layers(wsnet_s *n, int B, bool training = false) {
    const int64_t CK = static_cast<int64_t>(n->C) * 9 * n->C;
    for (int l = 0; l < n->L; ++l) {
        const float *bias = n->params.as<float>() + l * n->per_layer + CK;
        const __bf16 *X = bf(n->acts, l * n->max_batch * n->img);
        if (l + 1 < n->L)
            HIP_TRY(sgtv::wsn::conv_relu(X, bf(n->wf, l * CK), bias, B, n->H, n->W,
                                         bf(n->acts, (l + 1) * n->max_batch * n->img),
                                         training ? bf(n->xt, (l + 1) * 3 * n->max_batch * n->img) : nullptr,
                                         n->stream));
        else
            // training: only z (the loss kernel forms softplus(z) itself)
            HIP_TRY(sgtv::wsn::conv_softplus(X, bf(n->wf, l * CK), bias, B, n->H, n->W,
                                             n->z_last.as<float>(), training ? nullptr : n->out.as<float>(),
                                             n->stream));
    }
    return SGTV_OK;
}

int net_forward(wsnet_s *n, int B, bool training = false) {
    HIP_TRY(sgtv::wsn::to_bf16(n->xin.as<float>(), bf(n->acts), B * n->img, n->stream));
    return net_layers(n, B, training);
}

int net_check(wsnet_s *n, int B, int mk) {
    if (!n) return fail(SGTV_EINVAL, "null network");
    if (!n->have_params) return fail(SGTV_ESTATE, "no parameters set (call wsnet_set_params)");
    if (B < 1 || B > n->max_batch) return fail(SGTV_EINVAL, "batch must be in [1, max_batch]");
    return check_mem_kind(mk);
}

}  // namespace

extern "C" {

int64_t wsnet_param_count(int32_t layers, int32_t channels) {
    return static_cast<int64_t>(layers) * (static_cast<int64_t>(channels) * 9 * channels + channels);
}

int wsnet_create(wsnet *out, int device, void *hip_stream, int32_t layers, int32_t height,
                 int32_t width, int32_t channels, int32_t max_batch) {
    if (!out) return fail(SGTV_EINVAL, "out is NULL");
    if (channels != 64) return fail(SGTV_ESHAPE, "channels must be 64");
    if (width != 64) return fail(SGTV_ESHAPE, "width must be 64");
    if (height < 2 || height % 2 != 0) return fail(SGTV_ESHAPE, "height must be even and at least 2");
    if (layers < 1 || layers > 16) return fail(SGTV_EINVAL, "layers must be in [1, 16]");
    if (max_batch < 1 || max_batch > 4096) return fail(SGTV_EINVAL, "max_batch must be in [1, 4096]");
    int nd = 0;
    HIP_TRY(hipGetDeviceCount(&nd));
    if (device < 0 || device >= nd) return fail(SGTV_EINVAL, "device index out of range");
    DeviceGuard g(device);
    try {
        auto n = std::make_unique<wsnet_s>();
        n->device = device;
        n->stream = static_cast<hipStream_t>(hip_stream);
        n->L = layers; n->H = height; n->W = width; n->C = channels; n->max_batch = max_batch;
        n->per_layer = static_cast<int64_t>(channels) * 9 * channels + channels;
        n->n_param = wsnet_param_count(layers, channels);
        n->img = static_cast<int64_t>(height) * width * channels;
        const int64_t CK = static_cast<int64_t>(channels) * 9 * channels;
        const int64_t big = static_cast<int64_t>(max_batch) * n->img;
        HIP_TRY(n->params.alloc(sizeof(float) * n->n_param));
        HIP_TRY(n->grad.alloc(sizeof(float) * n->n_param));
        HIP_TRY(n->m.alloc(sizeof(float) * n->n_param));
        HIP_TRY(n->v.alloc(sizeof(float) * n->n_param));
        HIP_TRY(n->wf.alloc(2 * CK * layers));
        HIP_TRY(n->wb.alloc(2 * CK * layers));
        HIP_TRY(n->acts.alloc(2 * big * layers));
        HIP_TRY(n->z_last.alloc(sizeof(float) * big));
        HIP_TRY(n->out.alloc(sizeof(float) * big));
        HIP_TRY(n->xin.alloc(sizeof(float) * big));
        HIP_TRY(n->tgt.alloc(sizeof(float) * big));
        HIP_TRY(n->dz[0].alloc(2 * big));
        HIP_TRY(n->dz[1].alloc(2 * big));
        HIP_TRY(n->wpart.alloc(sizeof(float) * (CK + channels) * max_batch * (height / sgtv::wsn::wgrad_rows(height))));
        HIP_TRY(n->xt.alloc(2 * 3 * big * layers));
        HIP_TRY(n->dt.alloc(2 * big));
        HIP_TRY(n->lpart.alloc(sizeof(double) * kLossBlocks));
        HIP_TRY(n->lred.alloc(sizeof(double) * 4));
        HIP_TRY(n->lsum.alloc(sizeof(double) * 2));
        HIP_TRY(hipMemsetAsync(n->lsum.p, 0, sizeof(double) * 2, n->stream));
        HIP_TRY(n->ipart.alloc(sizeof(double) * kImageBlocks * max_batch));
        HIP_TRY(n->isum.alloc(sizeof(double) * max_batch));
        *out = n.release();
    } catch (const std::bad_alloc &) {
        return fail(SGTV_ENOMEM, "host allocation failed");
    }
    return SGTV_OK;
}

void wsnet_destroy(wsnet net) {
    if (!net) return;
    DeviceGuard g(net->device);
    if (net->stream) (void)hipStreamSynchronize(net->stream);
    else (void)hipDeviceSynchronize();
    delete net;
}

int wsnet_set_params(wsnet net, const float *params, int64_t n, int mem_kind) {
    if (!net || !params) return fail(SGTV_EINVAL, "null argument");
    if (int e = check_mem_kind(mem_kind)) return e;
    if (n != net->n_param) return fail(SGTV_ESHAPE, "parameter count does not match the network");
    DeviceGuard g(net->device);
    std::vector<float> h;
    HIP_TRY(hipStreamSynchronize(net->stream));
    HIP_TRY(fetch(h, params, n, mem_kind));
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(h[i])) return fail(SGTV_EINVAL, "parameters must be finite");
    HIP_TRY(hipMemcpyAsync(net->params.p, h.data(), sizeof(float) * n, hipMemcpyHostToDevice, net->stream));
    HIP_TRY(hipMemsetAsync(net->m.p, 0, sizeof(float) * n, net->stream));
    HIP_TRY(hipMemsetAsync(net->v.p, 0, sizeof(float) * n, net->stream));
    if (int e = net_weights(net)) return e;
    HIP_TRY(hipStreamSynchronize(net->stream));
    net->step = 0;
    net->have_params = true;
    net->have_grad = false;
    return SGTV_OK;
}

int wsnet_get_params(wsnet net, float *params, int64_t n, int mem_kind) {
    if (!net || !params) return fail(SGTV_EINVAL, "null argument");
    if (int e = check_mem_kind(mem_kind)) return e;
    if (n != net->n_param) return fail(SGTV_ESHAPE, "parameter count does not match the network");
    DeviceGuard g(net->device);
    HIP_TRY(hipMemcpyAsync(params, net->params.p, sizeof(float) * n, to_caller(mem_kind), net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    return SGTV_OK;
}

namespace {
struct WsnetFileHeader {
    char magic[4];          // "WSNT"
    int32_t version;        // 1
    int32_t layers, channels;
    int64_t n_params;       // FP32 values that follow, little endian
};
}  // namespace

int wsnet_save(wsnet net, const char *path) {
    if (!net || !path) return fail(SGTV_EINVAL, "null argument");
    if (!net->have_params) return fail(SGTV_ESTATE, "no parameters set (call wsnet_set_params)");
    std::vector<float> h(static_cast<size_t>(net->n_param));
    if (int e = wsnet_get_params(net, h.data(), net->n_param, SGTV_HOST)) return e;
    WsnetFileHeader hd{{'W', 'S', 'N', 'T'}, 1, net->L, net->C, net->n_param};
    std::FILE *fp = std::fopen(path, "wb");
    if (!fp) return fail(SGTV_EINVAL, "cannot open the file for writing");
    const bool ok = std::fwrite(&hd, sizeof(hd), 1, fp) == 1 &&
                    std::fwrite(h.data(), sizeof(float), h.size(), fp) == h.size();
    const bool closed = std::fclose(fp) == 0;
    if (!ok || !closed) return fail(SGTV_EINVAL, "writing the file failed");
    return SGTV_OK;
}

int wsnet_load(wsnet net, const char *path) {
    if (!net || !path) return fail(SGTV_EINVAL, "null argument");
    std::FILE *fp = std::fopen(path, "rb");
    if (!fp) return fail(SGTV_EINVAL, "cannot open the file for reading");
    WsnetFileHeader hd{};
    std::vector<float> h;
    bool ok = std::fread(&hd, sizeof(hd), 1, fp) == 1 && std::memcmp(hd.magic, "WSNT", 4) == 0 &&
              hd.version == 1;
    if (ok && (hd.layers != net->L || hd.channels != net->C || hd.n_params != net->n_param)) {
        std::fclose(fp);
        return fail(SGTV_ESHAPE, "the file holds a network of another shape");
    }
    if (ok) {
        h.resize(static_cast<size_t>(hd.n_params));
        ok = std::fread(h.data(), sizeof(float), h.size(), fp) == h.size();
    }
    std::fclose(fp);
    if (!ok) return fail(SGTV_EINVAL, "not a network file, or truncated");
    return wsnet_set_params(net, h.data(), net->n_param, SGTV_HOST);
}

int wsnet_forward(wsnet net, const float *x_in, int32_t batch, float *x0, int mem_kind) {
    if (int e = net_check(net, batch, mem_kind)) return e;
    if (!x_in || !x0) return fail(SGTV_EINVAL, "null argument");
    DeviceGuard g(net->device);
    const int64_t cnt = batch * net->img;
    if (int e = net_stage(net, net->xin, x_in, cnt, mem_kind)) return e;
    if (int e = net_forward(net, batch)) return e;
    HIP_TRY(hipMemcpyAsync(x0, net->out.p, sizeof(float) * cnt, to_caller(mem_kind), net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    return SGTV_OK;
}

int wsnet_start(wsnet net, const float *f, int32_t batch, int mode, double c_out, double floor, float *x0,
                int mem_kind) {
    if (int e = net_check(net, batch, mem_kind)) return e;
    if (!f || !x0) return fail(SGTV_EINVAL, "null argument");
    if (mode != WSNET_START_RATIO && mode != WSNET_START_DIRECT) return fail(SGTV_EINVAL, "unknown start mode");
    if (!(c_out > 0.0) || !std::isfinite(c_out)) return fail(SGTV_EINVAL, "c_out must be finite and > 0");
    if (!(floor >= 0.0) || !std::isfinite(floor)) return fail(SGTV_EINVAL, "floor must be finite and >= 0");
    DeviceGuard g(net->device);
    const int64_t cnt = batch * net->img;
    if (int e = net_stage(net, net->xin, f, cnt, mem_kind)) return e;
    HIP_TRY(sgtv::wsn::image_partials(net->xin.as<float>(), net->img, batch, kImageBlocks,
                                      net->ipart.as<double>(), net->stream));
    HIP_TRY(sgtv::launch_reduce(net->ipart.as<double>(), kImageBlocks, batch, net->isum.as<double>(), net->stream));
    HIP_TRY(sgtv::wsn::scale_to_bf16(net->xin.as<float>(), net->isum.as<double>(), net->img, cnt, bf(net->acts),
                                     net->stream));
    if (int e = net_layers(net, batch)) return e;
    HIP_TRY(sgtv::wsn::start_image(net->xin.as<float>(), net->out.as<float>(), net->isum.as<double>(), net->img,
                                   cnt, static_cast<float>(c_out), mode == WSNET_START_RATIO,
                                   static_cast<float>(floor), net->tgt.as<float>(), net->stream));
    HIP_TRY(hipMemcpyAsync(x0, net->tgt.p, sizeof(float) * cnt, to_caller(mem_kind), net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    return SGTV_OK;
}

}  // extern "C"

namespace {

// Forward and backward pass of a staged batch (inputs in xin, targets in
// tgt): the gradient in grad, the summed squared error in lred[0]; nothing
// waits for the device.
int net_backward(wsnet_s *net, int32_t batch) {
    const int64_t cnt = batch * net->img;
    const int64_t CK = static_cast<int64_t>(net->C) * 9 * net->C;
    if (int e = net_forward(net, batch, true)) return e;
    int cur = 0;
    HIP_TRY(sgtv::wsn::mse_grad(net->tgt.as<float>(), net->z_last.as<float>(), cnt, bf(net->dz[cur]),
                                net->lpart.as<double>(), kLossBlocks, net->stream));
    HIP_TRY(sgtv::launch_reduce(net->lpart.as<double>(), kLossBlocks, 1, net->lred.as<double>(), net->stream));
    for (int l = net->L - 1; l >= 0; --l) {
        const __bf16 *X = bf(net->acts, l * net->max_batch * net->img);
        // the forward pass wrote X's shifted copies for every layer but the first, and
        // below the last layer the backward-data convolution has written dZ channel-major
        float *xt = reinterpret_cast<float *>(bf(net->xt, l * 3 * net->max_batch * net->img));
        HIP_TRY(sgtv::wsn::conv_wgrad(X, bf(net->dz[cur]), batch, net->H, xt, net->dt.as<float>(),
                                      net->wpart.as<float>(), net->grad.as<float>() + l * net->per_layer, l > 0,
                                      l + 1 < net->L, net->stream));
        if (l == 0) break;
        HIP_TRY(sgtv::wsn::conv_masked(bf(net->dz[cur]), bf(net->wb, l * CK), batch, net->H, net->W, X,
                                       bf(net->dz[cur ^ 1]), bf(net->dt), net->stream));
        cur ^= 1;
    }
    net->have_grad = true;
    return SGTV_OK;
}

int check_adam(double lr, double beta1, double beta2, double eps) {
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(SGTV_EINVAL, "Adam needs lr > 0, 0 <= beta1, beta2 < 1 and eps > 0");
    return SGTV_OK;
}

// One Adam step on the gradient in grad (Kingma and Ba), then the bf16 weights.
int net_adam(wsnet_s *net, double lr, double beta1, double beta2, double eps) {
    net->step += 1;
    const double c1 = 1.0 - std::pow(beta1, static_cast<double>(net->step));
    const double c2 = 1.0 - std::pow(beta2, static_cast<double>(net->step));
    HIP_TRY(sgtv::wsn::adam(net->params.as<float>(), net->grad.as<float>(), net->m.as<float>(),
                            net->v.as<float>(), net->n_param, static_cast<float>(lr), static_cast<float>(beta1),
                            static_cast<float>(beta2), static_cast<float>(1.0 - beta1),
                            static_cast<float>(1.0 - beta2), static_cast<float>(eps), static_cast<float>(c1),
                            static_cast<float>(c2), net->stream));
    return net_weights(net);
}

}  // namespace

extern "C" {

int wsnet_backward(wsnet net, const float *x_in, const float *target, int32_t batch,
                   double *loss, float *grad, int mem_kind) {
    if (int e = net_check(net, batch, mem_kind)) return e;
    if (!x_in || !target) return fail(SGTV_EINVAL, "null argument");
    DeviceGuard g(net->device);
    const int64_t cnt = batch * net->img;
    if (int e = net_stage(net, net->xin, x_in, cnt, mem_kind)) return e;
    if (int e = net_stage(net, net->tgt, target, cnt, mem_kind)) return e;
    if (int e = net_backward(net, batch)) return e;
    double h = 0.0;
    HIP_TRY(hipMemcpyAsync(&h, net->lred.p, sizeof(double), hipMemcpyDeviceToHost, net->stream));
    if (grad)
        HIP_TRY(hipMemcpyAsync(grad, net->grad.p, sizeof(float) * net->n_param, to_caller(mem_kind), net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    if (loss) *loss = h / static_cast<double>(cnt);
    return SGTV_OK;
}

int wsnet_adam_step(wsnet net, double lr, double beta1, double beta2, double eps) {
    if (!net) return fail(SGTV_EINVAL, "null network");
    if (!net->have_grad) return fail(SGTV_ESTATE, "no gradient (call wsnet_backward first)");
    if (int e = check_adam(lr, beta1, beta2, eps)) return e;
    DeviceGuard g(net->device);
    return net_adam(net, lr, beta1, beta2, eps);
}

int wsnet_train_step(wsnet net, const float *x_in, const float *target, int32_t batch, double lr, double beta1,
                     double beta2, double eps, int mem_kind) {
    if (int e = net_check(net, batch, mem_kind)) return e;
    if (!x_in || !target) return fail(SGTV_EINVAL, "null argument");
    if (int e = check_adam(lr, beta1, beta2, eps)) return e;
    DeviceGuard g(net->device);
    const int64_t cnt = batch * net->img;
    if (int e = net_stage(net, net->xin, x_in, cnt, mem_kind)) return e;
    if (int e = net_stage(net, net->tgt, target, cnt, mem_kind)) return e;
    if (int e = net_backward(net, batch)) return e;
    HIP_TRY(sgtv::wsn::loss_accumulate(net->lred.as<double>(), static_cast<double>(cnt), net->lsum.as<double>(),
                                       net->stream));
    return net_adam(net, lr, beta1, beta2, eps);
}

int wsnet_loss_sum(wsnet net, double *sum, int64_t *steps, int reset) {
    if (!net || !sum) return fail(SGTV_EINVAL, "null argument");
    DeviceGuard g(net->device);
    double h[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(h, net->lsum.p, sizeof(h), hipMemcpyDeviceToHost, net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    if (reset) {
        HIP_TRY(hipMemsetAsync(net->lsum.p, 0, sizeof(h), net->stream));
        HIP_TRY(hipStreamSynchronize(net->stream));
    }
    *sum = h[0];
    if (steps) *steps = static_cast<int64_t>(h[1]);
    return SGTV_OK;
}

int wsnet_reset_adam(wsnet net) {
    if (!net) return fail(SGTV_EINVAL, "null network");
    DeviceGuard g(net->device);
    HIP_TRY(hipMemsetAsync(net->m.p, 0, sizeof(float) * net->n_param, net->stream));
    HIP_TRY(hipMemsetAsync(net->v.p, 0, sizeof(float) * net->n_param, net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    net->step = 0;
    return SGTV_OK;
}

}  // extern "C"
