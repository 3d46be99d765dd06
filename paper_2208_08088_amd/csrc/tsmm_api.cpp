// Host runtime of libtsmm: the C ABI declared in include/tsmm.h.
//
// It plays the part of the paper's runtime stage (Sec. III, Sec. IV-A):
// the packed handle is the pre-pack module's output with its header
// (Sec. IV-A.3: contiguous packed blocks plus a header that locates them);
// the plan is the execution plan (tile from the install-time table,
// checked against the capacity limits that Eqs. (2)-(3) express for CPU
// caches, here LDS and registers); execute launches the COMPUTE kernels.
// Every argument is validated before the first HIP call.
#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cinttypes>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "tsmm_internal.h"

using namespace tsmm;

namespace {

thread_local std::string g_err;

tsmm_status fail(tsmm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

tsmm_status hip_fail(hipError_t e, const char *what) {
    return fail(TSMM_ERROR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int log_level() {
    static int lvl = [] {
        const char *s = getenv("TSMM_LOG");
        return s ? atoi(s) : 0;
    }();
    return lvl;
}

// Device and pinned-host allocations of the library go through here.
// TSMM_FAIL_ALLOC (a comma-separated list of allocation names: pack,
// pack_a, workspace, batched) makes the named allocations fail as if the
// device were out of memory, so that the error paths can be exercised.
bool alloc_fails(const char *what) {
    const char *s = getenv("TSMM_FAIL_ALLOC");
    if (!s || !*s) return false;
    const size_t n = strlen(what);
    for (const char *p = s; *p;) {
        const char *e = strchr(p, ',');
        const size_t len = e ? (size_t)(e - p) : strlen(p);
        if (len == n && strncmp(p, what, n) == 0) return true;
        if (!e) break;
        p = e + 1;
    }
    return false;
}

hipError_t dev_malloc(void **ptr, size_t bytes, const char *what) {
    *ptr = nullptr;
    if (alloc_fails(what)) return hipErrorOutOfMemory;
    return hipMalloc(ptr, bytes);
}

hipError_t host_malloc_pinned(void **ptr, size_t bytes, const char *what) {
    *ptr = nullptr;
    if (alloc_fails(what)) return hipErrorOutOfMemory;
    return hipHostMalloc(ptr, bytes, hipHostMallocDefault);
}

bool valid_dtype(int d) { return d == TSMM_F64 || d == TSMM_F32 || d == TSMM_BF16; }
bool valid_layout(int l) { return l == TSMM_OP_N || l == TSMM_OP_T || l == TSMM_COLMAJOR; }
bool valid_mode(int m) { return m == TSMM_MODE_NATIVE || m == TSMM_MODE_BF16X3 || m == TSMM_MODE_BF16X6; }

const char *dtype_name(tsmm_dtype d) { return d == TSMM_F64 ? "f64" : d == TSMM_F32 ? "f32" : "bf16"; }
const char *mode_name(tsmm_mode m) {
    return m == TSMM_MODE_NATIVE ? "native" : m == TSMM_MODE_BF16X3 ? "bf16x3" : "bf16x6";
}
const char *kernel_name(int k) {
    switch (k) {
    case TSMM_KERNEL_SIMPLE: return "simple";
    case TSMM_KERNEL_STREAM: return "stream";
    case TSMM_KERNEL_SPLITK: return "splitk";
    case TSMM_KERNEL_SPLITBF16: return "splitbf16";
    case TSMM_KERNEL_VALU64: return "valu64";
    case TSMM_KERNEL_WIDE: return "wide";
    case TSMM_KERNEL_BATCHED: return "batched";
    case TSMM_KERNEL_SLAB: return "slab";
    case TSMM_KERNEL_COLMAJOR: return "colmajor";
    default: return "auto";
    }
}

int split_terms(tsmm_dtype d, tsmm_mode m) {
    if (d == TSMM_BF16) return 1;
    if (m == TSMM_MODE_BF16X3) return 2;
    if (m == TSMM_MODE_BF16X6) return 3;
    return 0;
}
int split_products(tsmm_dtype d, tsmm_mode m) {
    if (d == TSMM_BF16) return 1;
    return m == TSMM_MODE_BF16X3 ? 3 : 6;
}

// ------------------------------------------------------------ device caps

tsmm_status query_caps(tsmm_device_caps *caps, int *device) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(TSMM_ERROR_NO_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    static std::mutex mu;
    static std::map<int, tsmm_device_caps> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        hipDeviceProp_t p;
        e = hipGetDeviceProperties(&p, dev);
        if (e != hipSuccess) return fail(TSMM_ERROR_NO_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        tsmm_device_caps c{};
        c.compute_units = p.multiProcessorCount;
        c.lds_bytes_per_cu = (int32_t)p.maxSharedMemoryPerMultiProcessor;
        int arch = 0;
        if (sscanf(p.gcnArchName, "gfx%d", &arch) != 1) arch = 0;
        c.gcn_arch = arch;
        it = cache.emplace(dev, c).first;
    }
    *caps = it->second;
    *device = dev;
    if (caps->gcn_arch != 950)
        return fail(TSMM_ERROR_NO_DEVICE, "device %d is gfx%d; this library is built for gfx950", dev,
                    caps->gcn_arch);
    return TSMM_SUCCESS;
}

// ------------------------------------------------------------- tile table
//
// Text table written by the install-time autotuner, one entry per line:
//   <layout N|T> <dtype f64|f32|bf16> <mode native|bf16x3|bf16x6>
//   <kc> <nt> <mclass> : <kernel> <rows_per_wave> <waves_per_wg>
//   <wg_per_cu> <splitk> <nsplit>
// op N: kc = packed k class, nt = 16-column tiles class, mclass = row class.
// op T: kc = 16-row tiles of the output (m), nt = 16-column tiles (n),
//       mclass = class of the shared dimension.
// '#' starts a comment.  Three key lines say what the timings were taken
// on:
//   key arch gfx<N>        the device architecture
//   key hip <version>      hipRuntimeGetVersion() of the runtime
//   key libtsmm <version>  tsmm_version() of the library
// A table whose keys are missing or differ from the running library and
// runtime is not used (its tiles were timed for other code); entries apply
// only to plans for the keyed architecture.

// Tile-table layout "B": the entry of batched plans of one dtype (key
// fields kc, nt, mclass are 0).
constexpr int kLayoutBatched = 16;

struct TableKey {
    int layout, dtype, mode, kc, nt, mclass;
    bool operator<(const TableKey &o) const {
        return std::tie(layout, dtype, mode, kc, nt, mclass) <
               std::tie(o.layout, o.dtype, o.mode, o.kc, o.nt, o.mclass);
    }
};

struct Table {
    std::map<TableKey, tsmm_tile> entries;
    std::string path;
    bool loaded = false;
    std::string error;
    int arch = 0;  // from "key arch gfx<N>"
};

int hip_runtime_version() {
    int v = 0;
    if (hipRuntimeGetVersion(&v) != hipSuccess) v = 0;
    return v;
}

std::string library_dir() {
    Dl_info info;
    if (dladdr((void *)&tsmm_version, &info) && info.dli_fname) {
        std::string p = info.dli_fname;
        size_t s = p.find_last_of('/');
        if (s != std::string::npos) return p.substr(0, s);
    }
    return ".";
}

int parse_kernel(const std::string &s) {
    if (s == "simple") return TSMM_KERNEL_SIMPLE;
    if (s == "stream") return TSMM_KERNEL_STREAM;
    if (s == "splitk") return TSMM_KERNEL_SPLITK;
    if (s == "splitbf16") return TSMM_KERNEL_SPLITBF16;
    if (s == "valu64") return TSMM_KERNEL_VALU64;
    if (s == "wide") return TSMM_KERNEL_WIDE;
    if (s == "batched") return TSMM_KERNEL_BATCHED;
    if (s == "slab") return TSMM_KERNEL_SLAB;
    if (s == "colmajor") return TSMM_KERNEL_COLMAJOR;
    return -1;
}

bool parse_table_line(const std::string &line, TableKey *key, tsmm_tile *tile) {
    std::istringstream is(line);
    std::string lay, dt, md, colon, kern;
    if (!(is >> lay >> dt >> md >> key->kc >> key->nt >> key->mclass >> colon >> kern)) return false;
    if (colon != ":") return false;
    key->layout = lay == "N"   ? TSMM_OP_N
                  : lay == "T" ? TSMM_OP_T
                  : lay == "C" ? TSMM_COLMAJOR
                  : lay == "B" ? kLayoutBatched
                               : -1;
    key->dtype = dt == "f64" ? TSMM_F64 : dt == "f32" ? TSMM_F32 : dt == "bf16" ? TSMM_BF16 : -1;
    key->mode = md == "native" ? TSMM_MODE_NATIVE : md == "bf16x3" ? TSMM_MODE_BF16X3 : md == "bf16x6" ? TSMM_MODE_BF16X6 : -1;
    if (key->layout < 0 || key->dtype < 0 || key->mode < 0) return false;
    tsmm_tile t{};
    t.kernel = parse_kernel(kern);
    if (t.kernel < 0) return false;
    if (!(is >> t.rows_per_wave >> t.waves_per_wg >> t.wg_per_cu >> t.splitk >> t.nsplit)) return false;
    // batched entries carry the chunk size as a sixth field
    if (key->layout == kLayoutBatched && !(is >> t.chunk_rows)) return false;
    if ((key->layout == kLayoutBatched) != (t.kernel == TSMM_KERNEL_BATCHED)) return false;
    *tile = t;
    return true;
}

Table &table() {
    static Table tab;
    static std::once_flag once;
    std::call_once(once, [] {
        const char *env = getenv("TSMM_TILE_TABLE");
        tab.path = env ? env : library_dir() + "/tile_table.txt";
        std::ifstream f(tab.path);
        if (!f) {
            tab.error = "cannot open " + tab.path;
            return;
        }
        std::string line;
        int lineno = 0;
        long hip = -1, lib = -1;
        while (std::getline(f, line)) {
            ++lineno;
            size_t h = line.find('#');
            if (h != std::string::npos) line.resize(h);
            if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
            std::istringstream ks(line);
            std::string w0, w1, w2;
            if ((ks >> w0) && w0 == "key") {
                bool ok = static_cast<bool>(ks >> w1 >> w2);
                if (ok && w1 == "arch") ok = sscanf(w2.c_str(), "gfx%d", &tab.arch) == 1;
                else if (ok && w1 == "hip") hip = atol(w2.c_str());
                else if (ok && w1 == "libtsmm") lib = atol(w2.c_str());
                else ok = false;
                if (!ok) {
                    tab.error = tab.path + ":" + std::to_string(lineno) + ": malformed key line";
                    tab.entries.clear();
                    return;
                }
                continue;
            }
            TableKey k;
            tsmm_tile t;
            if (!parse_table_line(line, &k, &t)) {
                tab.error = tab.path + ":" + std::to_string(lineno) + ": malformed entry";
                tab.entries.clear();
                return;
            }
            tab.entries[k] = t;
        }
        char why[256] = "";
        if (tab.arch <= 0 || hip < 0 || lib < 0)
            snprintf(why, sizeof why, "%s has no key lines (arch, hip, libtsmm)", tab.path.c_str());
        else if (lib != tsmm_version())
            snprintf(why, sizeof why, "%s was tuned for libtsmm %ld, this is %d", tab.path.c_str(), lib,
                     (int)tsmm_version());
        else if (hip != hip_runtime_version())
            snprintf(why, sizeof why, "%s was tuned on HIP runtime %ld, this is %d", tab.path.c_str(), hip,
                     hip_runtime_version());
        if (why[0]) {
            tab.error = why;
            tab.entries.clear();
            if (log_level() >= 1) fprintf(stderr, "[tsmm] tile table not used: %s; built-in tiles\n", why);
            return;
        }
        tab.loaded = true;
    });
    return tab;
}

// Is the table usable for a plan on a device of this architecture?  The
// reason goes to tsmm_last_error when it is not.
bool table_usable(const tsmm_device_caps &caps) {
    Table &tab = table();
    if (!tab.loaded) return false;
    if (tab.arch != caps.gcn_arch) {
        static std::once_flag once;
        std::call_once(once, [&] {
            if (log_level() >= 1)
                fprintf(stderr, "[tsmm] tile table %s is for gfx%d, the plan's device is gfx%d; built-in tiles\n",
                        tab.path.c_str(), tab.arch, caps.gcn_arch);
        });
        return false;
    }
    return true;
}

std::string table_unusable_reason(const tsmm_device_caps &caps) {
    Table &tab = table();
    if (!tab.loaded) return tab.error;
    char buf[320];
    snprintf(buf, sizeof buf, "%s is for gfx%d, the plan's device is gfx%d", tab.path.c_str(), tab.arch,
             caps.gcn_arch);
    return buf;
}

int mclass_of(int64_t m) { return m < (1 << 16) ? 0 : (m < (1 << 21) ? 1 : 2); }

// -------------------------------------------------------------- planning

// Shapes the wide kernels serve (op N binary32, n = 128 or 256, k <= 256,
// k % 8 == 0); the packed handle then carries their image.
bool wide_shape(tsmm_layout layout, tsmm_dtype dtype, int64_t k, int64_t n) {
    return layout == TSMM_OP_N && dtype == TSMM_F32 && (n == 128 || n == 256) && k > 0 && k <= kMaxKC &&
           k % 8 == 0;
}
int wide_kc(int64_t k) { return std::max(64, kclass32(k)); }

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

constexpr size_t kLdsBudget = 128 * 1024;  // packed-B bytes a workgroup may keep in LDS

// Packed depth of the 16x16x4 fragment image: the k class, or for k past
// the classes a multiple of the slab depth (0: no image).
int64_t frag4_depth(int64_t k) {
    if (kclass4(k)) return kclass4(k);
    return k <= kSlabMaxK ? (k + kSlabK - 1) / kSlabK * kSlabK : 0;
}

// Shapes the k-slab kernel serves: op N binary64 / binary32 native, n <= 256,
// a fragment image whose depth is a multiple of the slab.
bool slab_ok(const tsmm_plan_s &p) {
    return p.layout == TSMM_OP_N && p.mode == TSMM_MODE_NATIVE && (p.dtype == TSMM_F64 || p.dtype == TSMM_F32) &&
           ntclass(p.n) > 0 && frag4_depth(p.k) % kSlabK == 0 && frag4_depth(p.k) > 0;
}

// Which kernel family serves (layout, dtype, mode, shape)?
// Column-major shapes the column-major kernel serves.
bool colmajor_ok(const tsmm_plan_s &p) {
    const int vw = p.dtype == TSMM_F64 ? 2 : 4;
    return p.layout == TSMM_COLMAJOR && p.mode == TSMM_MODE_NATIVE && (p.dtype == TSMM_F64 || p.dtype == TSMM_F32) &&
           kclass4(p.k) && ntclass(p.n) && p.m % vw == 0;
}

int natural_kernel(const tsmm_plan_s &p) {
    if (p.layout == TSMM_COLMAJOR) return colmajor_ok(p) ? TSMM_KERNEL_COLMAJOR : TSMM_KERNEL_SIMPLE;
    if (p.layout == TSMM_OP_T) return p.dtype == TSMM_F64 ? TSMM_KERNEL_SPLITK : TSMM_KERNEL_SIMPLE;
    if (p.dtype == TSMM_BF16 || p.mode != TSMM_MODE_NATIVE)
        return (kclass32(p.k) && ntclass(p.n)) ? TSMM_KERNEL_SPLITBF16 : TSMM_KERNEL_SIMPLE;
    if (kclass4(p.k) && ntclass(p.n)) return TSMM_KERNEL_STREAM;
    return slab_ok(p) ? TSMM_KERNEL_SLAB : TSMM_KERNEL_SIMPLE;
}

bool wide_ok(const tsmm_plan_s &p) { return wide_shape(p.layout, p.dtype, p.k, p.n); }
int wide_products(const tsmm_plan_s &p) { return p.mode == TSMM_MODE_NATIVE ? 0 : split_products(p.dtype, p.mode); }

// binary64 op N shapes the vector-ALU kernel can run
bool valu64_ok(const tsmm_plan_s &p) {
    return p.layout == TSMM_OP_N && p.dtype == TSMM_F64 && p.mode == TSMM_MODE_NATIVE && p.k > 0 && p.k % 8 == 0 &&
           p.n > 0 && p.n % 16 == 0 && p.k <= 8192;
}

// Can kernel family `kernel` run this plan?
bool eligible(const tsmm_plan_s &p, int kernel) {
    switch (kernel) {
    case TSMM_KERNEL_SIMPLE: return p.mode == TSMM_MODE_NATIVE;
    case TSMM_KERNEL_VALU64: return valu64_ok(p);
    case TSMM_KERNEL_WIDE: return wide_ok(p);
    case TSMM_KERNEL_SLAB: return slab_ok(p);
    case TSMM_KERNEL_COLMAJOR: return colmajor_ok(p);
    default: return kernel == natural_kernel(p);
    }
}

// Parts of the k range for the k-slab kernel: the row blocks alone fill
// the device in whole waves of workgroups when there are many of them;
// otherwise the smallest split (at most 16, at most one part per slab)
// whose items fill the last wave to 90%, else the best filled.
int slab_splitk(const tsmm_plan_s &p, int RT) {
    const int64_t cus = std::max(1, p.caps.compute_units);
    const int64_t nrb = (p.m + slab_rows(RT) - 1) / slab_rows(RT);
    const int64_t nsl = std::max<int64_t>(1, frag4_depth(p.k) / kSlabK);
    if (nrb >= 8 * cus) return 1;
    int best = 1;
    double best_fill = 0.0;
    for (int s = 1; s <= 16 && s <= nsl; ++s) {
        const int64_t items = nrb * s;
        const double fill = (double)items / (double)(((items + cus - 1) / cus) * cus);
        if (fill >= 0.9) return s;
        if (fill > best_fill + 1e-9) {
            best_fill = fill;
            best = s;
        }
    }
    return best;
}

int pow2_tiles(int64_t d) {  // 16-wide tiles of a small dimension, as 1, 2 or 4
    int t = (int)((d + 15) / 16);
    return t <= 1 ? 1 : (t <= 2 ? 2 : 4);
}

tsmm_tile default_tile(const tsmm_plan_s &p, int kernel) {
    tsmm_tile t{};
    t.kernel = kernel;
    t.waves_per_wg = 4;
    t.nsplit = 1;
    t.splitk = 1;
    switch (kernel) {
    case TSMM_KERNEL_STREAM: {
        const int KC = kclass4(p.k), NT = ntclass(p.n);
        const int w = KC * NT;
        const bool vec = vec_mapping(p.dtype, p.k, KC);
        // column groups: the smallest split whose B slice fits the LDS budget
        t.nsplit = 1;
        const int pg = frag4_pg(p.dtype, NT, p.n);  // column groups keep whole interleave groups
        while ((size_t)(KC / 4) * (NT / t.nsplit) * 64 * elem_bytes(p.dtype) > kLdsBudget && t.nsplit < NT / pg)
            t.nsplit *= 2;
        const int NTs = NT / t.nsplit;
        t.rows_per_wave = w <= 64 ? 4 : (w <= 256 ? 2 : 1);
        while (t.rows_per_wave > 1 && !stream_variant_exists(p.dtype, KC, NTs, t.rows_per_wave, vec, pg > 1))
            t.rows_per_wave /= 2;
        t.wg_per_cu = 8;
        break;
    }
    case TSMM_KERNEL_SPLITBF16: {
        const int KC = kclass32(p.k), NT = ntclass(p.n), terms = std::max(1, split_terms(p.dtype, p.mode));
        const int pg = bfrag_pg(p.dtype, NT, p.n);
        t.nsplit = 1;
        while ((size_t)(KC / 32) * (NT / t.nsplit) * terms * 64 * 16 > kLdsBudget && t.nsplit < NT / pg)
            t.nsplit *= 2;
        const int NTs = NT / t.nsplit;
        t.rows_per_wave = KC * NTs <= 1024 ? 2 : 1;
        while (t.rows_per_wave > 1 &&
               !splitbf16_variant_exists(p.dtype, KC, NTs, t.rows_per_wave, split_products(p.dtype, p.mode), pg > 1))
            t.rows_per_wave /= 2;
        t.wg_per_cu = 4;
        break;
    }
    case TSMM_KERNEL_VALU64:
        t.rows_per_wave = p.n % 32 == 0 ? 32 : 16;  // columns per wavefront
        t.wg_per_cu = 2;
        break;
    case TSMM_KERNEL_WIDE:
        // 32-row tiles: 256 accumulator registers (the split modes keep two)
        t.rows_per_wave = (p.n == 128 && p.mode == TSMM_MODE_NATIVE) ? 4 : 2;
        t.wg_per_cu = 1;
        break;
    case TSMM_KERNEL_COLMAJOR: {
        // column groups: at most 4 column tiles of C per wavefront (8 at
        // the k class 4; the accumulators of two or four m-tiles and, with
        // beta != 0, the C vectors read ahead) and a packed slice within
        // the LDS budget
        const int KC = kclass4(p.k), NT = ntclass(p.n);
        t.nsplit = 1;
        while ((NT / t.nsplit > (KC >= 8 ? 4 : 8) ||
                (size_t)(KC / 4) * (NT / t.nsplit) * 64 * elem_bytes(p.dtype) > kLdsBudget) &&
               t.nsplit < NT)
            t.nsplit *= 2;
        // rows_per_wave: column groups inside the workgroup.  Two groups of
        // wavefronts in one workgroup instead of two workgroups when both
        // slices fit the LDS: the second read of A then hits the cache.
        t.rows_per_wave = 1;
        if (t.nsplit == 2 && (size_t)(KC / 4) * NT * 64 * elem_bytes(p.dtype) <= kLdsBudget &&
            colmajor_variant_exists(p.dtype, KC, NT / 2, 2)) {
            t.rows_per_wave = 2;
            t.nsplit = 1;
        }
        t.wg_per_cu = 8;
        break;
    }
    case TSMM_KERNEL_SLAB: {
        // row tiles per wavefront: accumulators (RT * NT tiles of 8 or 4
        // registers) and two A register sets (2 * RT * 8 values) within
        // about 200 registers, at most 4
        const int NT = ntclass(p.n), regs = p.dtype == TSMM_F64 ? 8 : 4;
        t.rows_per_wave = 4;
        while (t.rows_per_wave > 1 && t.rows_per_wave * (NT * regs + 2 * 2 * regs) > 200) t.rows_per_wave /= 2;
        t.wg_per_cu = 1;
        t.splitk = slab_splitk(p, t.rows_per_wave);
        break;
    }
    case TSMM_KERNEL_SPLITK:
        t.rows_per_wave = 2;  // RG: 4-row groups per wavefront iteration
        t.wg_per_cu = 2;
        t.splitk = std::max<int64_t>(1, std::min<int64_t>(2 * (int64_t)p.caps.compute_units, (p.k + 255) / 256));
        break;
    default:
        t.rows_per_wave = 1;
        t.wg_per_cu = 1;
        break;
    }
    return t;
}

// Workgroups of a grid-stride op N launch: enough for the row tiles, at
// most wg_per_cu per compute unit; with column groups the row-block count is
// a multiple of 8 so that a row block's groups share an XCD.
int64_t row_grid(const tsmm_plan_s &p, const tsmm_tile &t, int64_t cus) {
    const int64_t waves = ((p.m + 15) / 16 + t.rows_per_wave - 1) / t.rows_per_wave;
    const int64_t wgs = (waves + t.waves_per_wg - 1) / t.waves_per_wg;
    int64_t rows = std::max<int64_t>(1, std::min<int64_t>(wgs, cus * t.wg_per_cu / t.nsplit));
    if (t.nsplit > 1) rows = (rows + 7) / 8 * 8;
    return rows * t.nsplit;
}

// Validate a tile for the plan and derive the launch geometry.
tsmm_status apply_tile(tsmm_plan_s &p, const tsmm_tile &tile_in) {
    tsmm_tile t = tile_in;
    if (t.kernel == TSMM_KERNEL_AUTO) t.kernel = natural_kernel(p);
    if (!eligible(p, t.kernel)) {
        if (t.kernel == TSMM_KERNEL_SIMPLE)
            return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes need k <= %d and n <= 256", kMaxKC);
        return fail(TSMM_ERROR_NOT_SUPPORTED, "kernel %s cannot run this plan (natural kernel %s)",
                    kernel_name(t.kernel), kernel_name(natural_kernel(p)));
    }
    tsmm_tile d = default_tile(p, t.kernel);
    if (t.rows_per_wave == 0) t.rows_per_wave = d.rows_per_wave;
    if (t.waves_per_wg == 0) t.waves_per_wg = d.waves_per_wg;
    if (t.wg_per_cu == 0) t.wg_per_cu = d.wg_per_cu;
    if (t.splitk == 0) t.splitk = d.splitk;
    if (t.nsplit == 0) t.nsplit = d.nsplit;
    // eight wavefronts only for the wide kernel (two per SIMD)
    const int max_waves = t.kernel == TSMM_KERNEL_WIDE ? 8 : 4;
    if (t.rows_per_wave < 0 || t.waves_per_wg < 1 || t.waves_per_wg > max_waves || !is_pow2(t.waves_per_wg) ||
        t.wg_per_cu < 1 || t.wg_per_cu > 32 || t.splitk < 1 || t.splitk > 65536 || t.nsplit < 1 ||
        t.nsplit > 16 || !is_pow2(t.nsplit))
        return fail(TSMM_ERROR_INVALID_VALUE, "tile out of range (waves_per_wg 1/2/4 (wide: 4/8), wg_per_cu 1..32, "
                                              "splitk 1..65536, nsplit 1/2/4/8/16)");
    if (t.nsplit > 1 && t.kernel != TSMM_KERNEL_STREAM && t.kernel != TSMM_KERNEL_SPLITBF16 &&
        t.kernel != TSMM_KERNEL_COLMAJOR)
        return fail(TSMM_ERROR_INVALID_VALUE, "nsplit applies to the op N fragment kernels only");
    const int64_t cus = std::max(1, p.caps.compute_units);
    p.block = 64 * t.waves_per_wg;
    p.workspace_bytes = 0;
    p.grid_y = 1;
    switch (t.kernel) {
    case TSMM_KERNEL_STREAM: {
        p.KC = kclass4(p.k);
        p.NT = ntclass(p.n);
        p.vec = vec_mapping(p.dtype, p.k, p.KC);
        if (t.nsplit > p.NT) return fail(TSMM_ERROR_INVALID_VALUE, "nsplit %d > %d column tiles", t.nsplit, p.NT);
        const int NTs = p.NT / t.nsplit;
        const int pg = frag4_pg(p.dtype, p.NT, p.n);
        if (NTs % pg != 0)
            return fail(TSMM_ERROR_INVALID_VALUE, "nsplit %d splits the %d-tile column interleave groups", t.nsplit,
                        pg);
        if (!stream_variant_exists(p.dtype, p.KC, NTs, t.rows_per_wave, p.vec, pg > 1))
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no stream kernel for KC=%d NT=%d RT=%d vec=%d", p.KC, NTs,
                        t.rows_per_wave, (int)p.vec);
        // Eq. (2) analogue: the workgroup's slice of packed B must fit the LDS
        const size_t lds = (size_t)(p.KC / 4) * NTs * 64 * elem_bytes(p.dtype);
        if (lds <= kLdsBudget && (int64_t)lds > p.caps.lds_bytes_per_cu)
            return fail(TSMM_ERROR_NOT_SUPPORTED, "packed B slice (%zu bytes) exceeds LDS", lds);
        p.grid = row_grid(p, t, cus);
        break;
    }
    case TSMM_KERNEL_SPLITBF16: {
        p.KC = kclass32(p.k);
        p.NT = ntclass(p.n);
        p.vec = false;
        if (t.nsplit > p.NT) return fail(TSMM_ERROR_INVALID_VALUE, "nsplit %d > %d column tiles", t.nsplit, p.NT);
        const int NTs = p.NT / t.nsplit;
        const int pg = bfrag_pg(p.dtype, p.NT, p.n);
        if (NTs % pg != 0)
            return fail(TSMM_ERROR_INVALID_VALUE, "nsplit %d splits the %d-tile column interleave groups", t.nsplit,
                        pg);
        if (!splitbf16_variant_exists(p.dtype, p.KC, NTs, t.rows_per_wave, split_products(p.dtype, p.mode), pg > 1))
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no split-bf16 kernel for KC=%d NT=%d RT=%d", p.KC, NTs,
                        t.rows_per_wave);
        p.grid = row_grid(p, t, cus);
        break;
    }
    case TSMM_KERNEL_VALU64: {
        const int NB = t.rows_per_wave;
        if (!valu64_variant_exists(NB) || p.n % NB != 0)
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no vector-ALU kernel with %d columns per wavefront for n=%" PRId64,
                        NB, p.n);
        if (t.waves_per_wg != 4 || t.nsplit != 1)
            return fail(TSMM_ERROR_INVALID_VALUE, "the vector-ALU kernel runs 4 wavefronts and no column split");
        p.KC = kclass4(p.k);
        p.NT = ntclass(p.n);
        p.vec = false;
        const int64_t ncg = p.n / NB;
        p.grid_y = (ncg + 3) / 4;
        const int64_t tiles = (p.m + 63) / 64;
        p.grid = std::max<int64_t>(1, std::min<int64_t>(tiles, std::max<int64_t>(1, cus * t.wg_per_cu / p.grid_y)));
        break;
    }
    case TSMM_KERNEL_WIDE: {
        p.KC = wide_kc(p.k);
        p.NT = (int)(p.n / 32);
        p.vec = true;
        if ((t.waves_per_wg != 4 && t.waves_per_wg != 8) || t.wg_per_cu != 1 || t.nsplit != 1)
            return fail(TSMM_ERROR_INVALID_VALUE,
                        "the wide kernel runs one workgroup of 4 or 8 wavefronts per compute unit, no column split");
        if (!wide_variant_exists(wide_products(p), p.KC, p.NT, t.rows_per_wave, t.waves_per_wg))
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no wide kernel for KC=%d n=%" PRId64 " RT=%d waves=%d", p.KC,
                        p.n, t.rows_per_wave, t.waves_per_wg);
        const int64_t rows_wg = wide_rows_per_wg(t.rows_per_wave, t.waves_per_wg);
        const int64_t tiles = (p.m + rows_wg - 1) / rows_wg;
        p.grid = std::max<int64_t>(1, std::min<int64_t>(tiles, cus));
        break;
    }
    case TSMM_KERNEL_COLMAJOR: {
        p.KC = kclass4(p.k);
        p.NT = ntclass(p.n);
        p.vec = false;
        const int NG = t.rows_per_wave;  // column groups inside a workgroup
        if (NG != 1 && NG != 2)
            return fail(TSMM_ERROR_INVALID_VALUE, "column-major: rows_per_wave (column groups per workgroup) 1 or 2");
        if (t.nsplit * NG > p.NT)
            return fail(TSMM_ERROR_INVALID_VALUE, "nsplit %d x %d groups > %d column tiles", t.nsplit, NG, p.NT);
        const int NTw = p.NT / (t.nsplit * NG);
        if (!colmajor_variant_exists(p.dtype, p.KC, NTw, NG))
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no column-major kernel for KC=%d NT=%d groups=%d", p.KC, NTw,
                        NG);
        if (t.waves_per_wg != 4)
            return fail(TSMM_ERROR_INVALID_VALUE, "the column-major kernel runs 4 wavefronts per workgroup");
        // column blocks of 16 * VW m indices, one per wavefront step of each group
        const int vw = p.dtype == TSMM_F64 ? 2 : 4;
        const int64_t blocks = (p.m + 16 * vw - 1) / (16 * vw);
        const int64_t wgs = (blocks + t.waves_per_wg / NG - 1) / (t.waves_per_wg / NG);
        int64_t rows = std::max<int64_t>(1, std::min<int64_t>(wgs, cus * t.wg_per_cu / t.nsplit));
        if (t.nsplit > 1) rows = (rows + 7) / 8 * 8;
        p.grid = rows * t.nsplit;
        break;
    }
    case TSMM_KERNEL_SLAB: {
        const int64_t depth = frag4_depth(p.k);
        p.KC = (int)depth;
        p.NT = ntclass(p.n);
        p.vec = vec_mapping(p.dtype, p.k, p.KC);
        const bool il = frag4_pg(p.dtype, p.NT, p.n) > 1;
        if (!slab_variant_exists(p.dtype, p.NT, t.rows_per_wave, p.vec, il))
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no k-slab kernel for NT=%d RT=%d", p.NT, t.rows_per_wave);
        if (t.waves_per_wg != 4 || t.wg_per_cu != 1 || t.nsplit != 1)
            return fail(TSMM_ERROR_INVALID_VALUE,
                        "the k-slab kernel runs one workgroup of 4 wavefronts per compute unit, no column split");
        const int64_t nsl = depth / kSlabK;
        if (t.splitk > nsl || t.splitk > 64)
            return fail(TSMM_ERROR_INVALID_VALUE, "splitk %d: at most 64 and at most one part per 32-k slab (%" PRId64
                                                  ")", t.splitk, nsl);
        // the slab double buffer, the Eq. (2) analogue
        const size_t lds = 2 * (size_t)(kSlabK / 4) * p.NT * 64 * elem_bytes(p.dtype);
        if ((int64_t)lds > p.caps.lds_bytes_per_cu)
            return fail(TSMM_ERROR_NOT_SUPPORTED, "two slabs of packed B (%zu bytes) exceed LDS", lds);
        const int64_t nrb = (p.m + slab_rows(t.rows_per_wave) - 1) / slab_rows(t.rows_per_wave);
        p.grid = std::max<int64_t>(1, std::min<int64_t>(nrb * t.splitk, cus));
        if (t.splitk > 1)
            p.workspace_bytes = (size_t)t.splitk * (size_t)((p.m + 15) / 16) * p.NT * 64 * 4 * sizeof(double);
        break;
    }
    case TSMM_KERNEL_SPLITK: {
        const int MT = pow2_tiles(p.m), NT = pow2_tiles(p.n);
        if (!splitk_variant_exists(MT, NT, t.rows_per_wave))
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no split-k kernel for MT=%d NT=%d RG=%d", MT, NT,
                        t.rows_per_wave);
        p.KC = MT;
        p.NT = NT;
        p.grid = t.splitk;
        p.grid_y = ((p.m + 16 * MT - 1) / (16 * MT)) * ((p.n + 16 * NT - 1) / (16 * NT));
        p.workspace_bytes = (size_t)t.splitk * (size_t)p.m * (size_t)p.n * sizeof(double);
        break;
    }
    default:
        t.kernel = TSMM_KERNEL_SIMPLE;
        p.grid = std::max<int64_t>(1, (p.m * p.n + 255) / 256);
        p.block = 256;
        break;
    }
    p.tile = t;
    return TSMM_SUCCESS;
}

// ------------------------------------------------------ batched tiles

bool valid_chunk_rows(int c) { return c >= kBatchChunkMin && c <= kBatchChunkMax && is_pow2(c); }

// Workgroups per compute unit a batched plan can keep resident: 1, 2 or
// 4, as far as the LDS holds that many copies of the largest packed B.
bool batched_wpc_fits(const tsmm_plan_s &p, int wpc) {
    return (wpc == 1 || wpc == 2 || wpc == 4) && (int64_t)wpc * (int64_t)(p.batch_lds + 1024) <= p.caps.lds_bytes_per_cu;
}

// Chunk size and workgroups per CU of batched plans of `dtype`: the
// table's batched entry, else the defaults (one workgroup per CU).
int batched_table_chunk(tsmm_dtype dtype, const tsmm_device_caps &caps, bool *from_table, int *wpc = nullptr) {
    *from_table = false;
    if (wpc) *wpc = 1;
    Table &tab = table();
    if (table_usable(caps)) {
        auto it = tab.entries.find(TableKey{kLayoutBatched, dtype, TSMM_MODE_NATIVE, 0, 0, 0});
        if (it != tab.entries.end() && valid_chunk_rows(it->second.chunk_rows)) {
            *from_table = true;
            if (wpc) *wpc = it->second.wg_per_cu;
            return it->second.chunk_rows;
        }
    }
    return kBatchChunkDefault;
}

// Cut the instances (in execution order) into chunks (batch_instance_chunk
// rows each):
// the prefix of chunk counts goes to the device (synchronously) and the
// grid follows the work.
tsmm_status batched_chunks(tsmm_plan_s &p, int chunk_rows) {
    const size_t count = p.inst.size();
    std::vector<int64_t> inst_start(count + 1, 0);
    for (size_t e = 0; e < count; ++e) {
        const BatchedInstance &I = p.inst[p.order[e]];
        const int cr = batch_instance_chunk(chunk_rows, I.k, I.n, (int)elem_bytes(p.dtype));
        inst_start[e + 1] = inst_start[e] + (I.m + cr - 1) / cr;
    }
    if (inst_start[count] >= (int64_t)1 << 31) return fail(TSMM_ERROR_NOT_SUPPORTED, "batch too large (2^31 chunks)");
    hipError_t e = hipMemcpy(p.d_inst_start, inst_start.data(), sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batched chunk list upload");
    p.n_work = inst_start[count];
    p.tile.chunk_rows = chunk_rows;
    p.grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)p.caps.compute_units * p.tile.wg_per_cu, p.n_work));
    return TSMM_SUCCESS;
}

// tsmm_plan_set_tile on a batched plan: the chunk size and the workgroups
// per compute unit are free.
tsmm_status set_batched_tile(tsmm_plan_s &p, const tsmm_tile &t) {
    if (t.kernel != TSMM_KERNEL_AUTO && t.kernel != TSMM_KERNEL_BATCHED)
        return fail(TSMM_ERROR_NOT_SUPPORTED, "batched plans run the batched kernel");
    if ((t.rows_per_wave != 0) || (t.waves_per_wg != 0 && t.waves_per_wg != kBatchWaves) ||
        (t.splitk != 0 && t.splitk != 1) || (t.nsplit != 0 && t.nsplit != 1))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "batched plans take only chunk_rows and wg_per_cu (%d waves)",
                    kBatchWaves);
    bool from_table = false;
    int table_wpc = 1;
    const int chunk = t.chunk_rows ? t.chunk_rows : batched_table_chunk(p.dtype, p.caps, &from_table, &table_wpc);
    if (!valid_chunk_rows(chunk))
        return fail(TSMM_ERROR_INVALID_VALUE, "chunk_rows %d: a power of two in %d..%d", chunk, kBatchChunkMin,
                    kBatchChunkMax);
    // wg_per_cu 0: the table's with the table's chunk size, else the plan's current one
    const int wpc = t.wg_per_cu ? t.wg_per_cu
                                : t.chunk_rows ? p.tile.wg_per_cu
                                               : (from_table && batched_wpc_fits(p, table_wpc) ? table_wpc : 1);
    if (!batched_wpc_fits(p, wpc))
        return fail(TSMM_ERROR_INVALID_VALUE, "wg_per_cu %d: 1, 2 or 4 workgroups of %zu LDS bytes within %d", wpc,
                    p.batch_lds, p.caps.lds_bytes_per_cu);
    if (p.graphs > 0) return fail(TSMM_ERROR_INVALID_VALUE, "a graph captured from this plan still exists");
    hipError_t e = hipSetDevice(p.device);
    if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
    if (e != hipSuccess) return hip_fail(e, "batched plan re-tile");
    p.tile.wg_per_cu = wpc;
    tsmm_status st = batched_chunks(p, chunk);
    if (st != TSMM_SUCCESS) return st;
    p.tile_from_table = from_table;
    if (p.bound) {  // the bound descriptors carry each instance's chunk rows
        for (size_t e2 = 0; e2 < p.bound_desc.size(); ++e2) {
            const BatchedInstance &I = p.inst[p.order[e2]];
            p.bound_desc[e2].chunk_rows = batch_instance_chunk(chunk, I.k, I.n, (int)elem_bytes(p.dtype));
        }
        e = hipMemcpy(p.d_desc, p.bound_desc.data(), sizeof(BatchDesc) * p.bound_desc.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "batched descriptor update");
    }
    return TSMM_SUCCESS;
}

// The tile-table key of a plan's shape class.
TableKey plan_key(const tsmm_plan_s &p) {
    TableKey key{};
    key.layout = p.layout;
    key.dtype = p.dtype;
    key.mode = p.mode;
    if (p.layout != TSMM_OP_T) {
        key.kc = natural_kernel(p) == TSMM_KERNEL_SPLITBF16 ? kclass32(p.k) : kclass4(p.k);
        key.nt = ntclass(p.n);
        key.mclass = mclass_of(p.m);
    } else {
        key.kc = pow2_tiles(p.m);
        key.nt = pow2_tiles(p.n);
        key.mclass = mclass_of(p.k);
    }
    return key;
}

// Tiles the runtime evaluator (tsmm_plan_tune) chose in this process, by
// shape class; they take precedence over the tile table.
struct RuntimeCache {
    std::mutex mu;
    std::map<TableKey, tsmm_tile> entries;
};
RuntimeCache &runtime_cache() {
    static RuntimeCache c;
    return c;
}

tsmm_status choose_tile(tsmm_plan_s &p) {
    const int nat = natural_kernel(p);
    Table &tab = table();
    p.tile_from_table = 0;
    {
        RuntimeCache &rc = runtime_cache();
        std::lock_guard<std::mutex> lock(rc.mu);
        auto it = rc.entries.find(plan_key(p));
        if (it != rc.entries.end() && eligible(p, it->second.kernel)) {
            tsmm_plan_s trial = p;
            if (apply_tile(trial, it->second) == TSMM_SUCCESS) {
                p = trial;
                p.tile_from_table = 2;
                return TSMM_SUCCESS;
            }
            g_err.clear();
        }
    }
    if (table_usable(p.caps)) {
        const TableKey key = plan_key(p);
        auto it = tab.entries.find(key);
        if (it != tab.entries.end() && eligible(p, it->second.kernel)) {
            tsmm_plan_s trial = p;
            if (apply_tile(trial, it->second) == TSMM_SUCCESS) {
                p = trial;
                p.tile_from_table = true;
                return TSMM_SUCCESS;
            }
            if (log_level() >= 1)
                fprintf(stderr, "[tsmm] table entry rejected (%s); using the default tile\n", g_err.c_str());
        }
    } else if (getenv("TSMM_STRICT_TABLE")) {
        return fail(TSMM_ERROR_TABLE, "tile table: %s", table_unusable_reason(p.caps).c_str());
    } else if (log_level() >= 2) {
        fprintf(stderr, "[tsmm] tile table not used: %s\n", table_unusable_reason(p.caps).c_str());
    }
    // no table entry: the wide kernels where they apply (they read and split
    // A once at any n), else the natural family
    tsmm_tile t{};
    t.kernel = wide_ok(p) ? TSMM_KERNEL_WIDE : nat;
    return apply_tile(p, t);
}

tsmm_status make_plan(int64_t m, int64_t n, int64_t k, tsmm_layout layout, tsmm_dtype dtype,
                      const tsmm_device_caps *caps, int device, tsmm_plan_t *out) {
    std::unique_ptr<tsmm_plan_s> p(new (std::nothrow) tsmm_plan_s());
    if (!p) return fail(TSMM_ERROR_OUT_OF_MEMORY, "host allocation failed");
    p->m = m;
    p->n = n;
    p->k = k;
    p->layout = layout;
    p->dtype = dtype;
    p->mode = TSMM_MODE_NATIVE;
    p->caps = *caps;
    p->device = device;
    tsmm_status st = choose_tile(*p);
    if (st != TSMM_SUCCESS) return st;
    if (log_level() >= 1) {
        char buf[256];
        tsmm_plan_describe(p.get(), buf, sizeof buf);
        fprintf(stderr, "[tsmm] plan %s\n", buf);
    }
    *out = p.release();
    return TSMM_SUCCESS;
}

tsmm_status check_plan_args(int64_t m, int64_t n, int64_t k, int layout, int dtype, const void *out) {
    if (!out) return fail(TSMM_ERROR_INVALID_VALUE, "out is NULL");
    if (m < 0 || n < 0 || k < 0) return fail(TSMM_ERROR_INVALID_VALUE, "negative size");
    if (!valid_layout(layout)) return fail(TSMM_ERROR_INVALID_VALUE, "bad layout %d", layout);
    if (!valid_dtype(dtype)) return fail(TSMM_ERROR_INVALID_VALUE, "bad dtype %d", dtype);
    if (m > (INT64_C(1) << 40) || n > (INT64_C(1) << 30) || k > (INT64_C(1) << 40))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "size beyond the library's index range");
    if (layout != TSMM_OP_T && (n > INT32_MAX || k > INT32_MAX))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "op N and column-major need n, k < 2^31");
    if (layout == TSMM_COLMAJOR && dtype == TSMM_BF16)
        return fail(TSMM_ERROR_NOT_SUPPORTED, "column-major operands take binary64 or binary32");
    if (layout == TSMM_OP_T && (m > INT32_MAX || n > INT32_MAX))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "op T needs m, n < 2^31");
    return TSMM_SUCCESS;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

const char *tsmm_status_string(tsmm_status s) {
    switch (s) {
    case TSMM_SUCCESS: return "success";
    case TSMM_ERROR_INVALID_VALUE: return "invalid value";
    case TSMM_ERROR_SHAPE_MISMATCH: return "plan and packed operand do not match";
    case TSMM_ERROR_NOT_SUPPORTED: return "not supported";
    case TSMM_ERROR_TABLE: return "tile table error";
    case TSMM_ERROR_OUT_OF_MEMORY: return "out of memory";
    case TSMM_ERROR_NO_DEVICE: return "no usable device";
    case TSMM_ERROR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *tsmm_last_error(void) { return g_err.c_str(); }

int32_t tsmm_version(void) { return 10100; }

tsmm_status tsmm_table_key(int32_t gcn_arch, char *buf, size_t len) {
    g_err.clear();
    if (!buf || len == 0) return fail(TSMM_ERROR_INVALID_VALUE, "NULL buffer");
    if (gcn_arch < 0) return fail(TSMM_ERROR_INVALID_VALUE, "bad architecture %d", (int)gcn_arch);
    if (gcn_arch == 0) {
        tsmm_device_caps caps;
        int dev = 0;
        const tsmm_status st = query_caps(&caps, &dev);
        if (st != TSMM_SUCCESS) return st;
        gcn_arch = caps.gcn_arch;
    }
    const int n = snprintf(buf, len, "key arch gfx%d\nkey hip %d\nkey libtsmm %d\n", (int)gcn_arch,
                           hip_runtime_version(), (int)tsmm_version());
    if (n < 0 || (size_t)n >= len) return fail(TSMM_ERROR_INVALID_VALUE, "buffer of %zu bytes is too small", len);
    return TSMM_SUCCESS;
}

// ------------------------------------------------------------------ pack

tsmm_status tsmm_pack(const void *B, int64_t k, int64_t n, tsmm_layout layout, tsmm_dtype dtype,
                      tsmm_mode mode, void *stream, tsmm_packed_t *out) {
    g_err.clear();
    if (!out) return fail(TSMM_ERROR_INVALID_VALUE, "out is NULL");
    *out = nullptr;
    if (k < 0 || n < 0) return fail(TSMM_ERROR_INVALID_VALUE, "negative size");
    if (!valid_layout(layout)) return fail(TSMM_ERROR_INVALID_VALUE, "bad layout %d", (int)layout);
    if (!valid_dtype(dtype)) return fail(TSMM_ERROR_INVALID_VALUE, "bad dtype %d", (int)dtype);
    if (!valid_mode(mode)) return fail(TSMM_ERROR_INVALID_VALUE, "bad mode %d", (int)mode);
    if (mode != TSMM_MODE_NATIVE && (dtype != TSMM_F32 || layout != TSMM_OP_N))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes take op N binary32 operands");
    if (layout == TSMM_COLMAJOR && dtype == TSMM_BF16)
        return fail(TSMM_ERROR_NOT_SUPPORTED, "column-major operands take binary64 or binary32");
    if (k * n > 0 && !B) return fail(TSMM_ERROR_INVALID_VALUE, "B is NULL");
    if (k > INT32_MAX || n > INT32_MAX) return fail(TSMM_ERROR_NOT_SUPPORTED, "k, n must be < 2^31");
    const int terms = split_terms(dtype, mode);
    if (mode != TSMM_MODE_NATIVE && (!kclass32(k) || !ntclass(n)))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes need k <= %d and n <= 256", kMaxKC);

    std::unique_ptr<tsmm_packed_s> P(new (std::nothrow) tsmm_packed_s());
    if (!P) return fail(TSMM_ERROR_OUT_OF_MEMORY, "host allocation failed");
    P->k = k;
    P->n = n;
    P->layout = layout;
    P->dtype = dtype;
    P->mode = mode;
    if (layout == TSMM_OP_T || k == 0 || n == 0) {  // nothing to copy
        P->ref = B;
        *out = P.release();
        return TSMM_SUCCESS;
    }
    PackedLayout &L = P->L;
    const size_t eb = elem_bytes(dtype);
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    L.off_rowmajor = off;
    off = align(off + (size_t)k * n * eb);
    if (terms > 0) {  // bf16 fragments (split planes or plain bf16)
        L.KC = kclass32(k);
        L.NT = ntclass(n);
        L.terms = terms;
        L.pg = bfrag_pg(dtype, L.NT, n);
        if (L.KC && L.NT) {
            L.off_frag = off;
            off = align(off + (size_t)L.KC * L.NT * 16 * terms * 2);
        }
        if (mode != TSMM_MODE_NATIVE) {
            L.off_planes = off;
            off = align(off + (size_t)terms * k * n * 2);
            L.off_exps = off;
            off = align(off + (size_t)n * 4);
        }
    } else if (layout == TSMM_COLMAJOR) {
        // the column-major kernel: scalar k-slot mapping (A's columns are
        // separate streams), plain column order
        L.KC = kclass4(k);
        L.NT = ntclass(n);
        if (L.KC && L.NT) {
            L.off_frag = off;
            off = align(off + (size_t)L.KC * L.NT * 16 * eb);
        }
    } else {
        L.KC = (int)frag4_depth(k);
        L.NT = ntclass(n);
        if (L.KC && L.NT) {
            L.vec = vec_mapping(dtype, k, L.KC);
            L.pg = frag4_pg(dtype, L.NT, n);
            L.off_frag = off;
            off = align(off + (size_t)L.KC * L.NT * 16 * eb);
        }
    }
    if (wide_shape(layout, dtype, k, n)) {
        L.wide_KC = wide_kc(k);
        L.wide_NT = (int)(n / 32);
        L.off_wide = off;
        off = align(off + wide_image_bytes(L.wide_KC, L.wide_NT, terms));
    }
    L.bytes = off;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(TSMM_ERROR_NO_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    P->device = dev;
    e = dev_malloc(&P->dev, L.bytes, "pack");
    if (e != hipSuccess) return fail(TSMM_ERROR_OUT_OF_MEMORY, "hipMalloc(%zu): %s", L.bytes, hipGetErrorString(e));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(P->dev);
    e = hipMemcpyAsync(base + L.off_rowmajor, B, (size_t)k * n * eb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && L.KC && L.NT) {
        if (terms > 0)
            e = launch_pack_bf16(dtype, B, base + L.off_frag,
                                 mode != TSMM_MODE_NATIVE ? base + L.off_planes : nullptr,
                                 mode != TSMM_MODE_NATIVE ? reinterpret_cast<int32_t *>(base + L.off_exps) : nullptr,
                                 k, n, L.KC, L.NT, terms, L.pg, s);
        else
            e = launch_pack_frag4(dtype, layout == TSMM_COLMAJOR, B, base + L.off_frag, k, n, L.KC, L.NT, L.vec,
                                  L.pg, s);
    }
    if (e == hipSuccess && L.wide_KC)  // after the split planes it reads
        e = launch_pack_wide(B, terms > 0 ? base + L.off_planes : nullptr, base + L.off_wide, k, n, L.wide_KC,
                             L.wide_NT, terms, s);
    if (e != hipSuccess) {
        (void)hipFree(P->dev);
        return hip_fail(e, "pack");
    }
    *out = P.release();
    return TSMM_SUCCESS;
}

tsmm_status tsmm_packed_bytes(tsmm_packed_t p, size_t *bytes) {
    g_err.clear();
    if (!p || !bytes) return fail(TSMM_ERROR_INVALID_VALUE, "NULL argument");
    *bytes = p->dev ? p->L.bytes : 0;
    return TSMM_SUCCESS;
}

tsmm_status tsmm_unpack(tsmm_packed_t p, void *B_out, void *stream) {
    g_err.clear();
    if (!p) return fail(TSMM_ERROR_INVALID_VALUE, "packed is NULL");
    if (p->is_a) return fail(TSMM_ERROR_NOT_SUPPORTED, "packed A handles are not unpacked");
    if (p->layout == TSMM_OP_T) return fail(TSMM_ERROR_NOT_SUPPORTED, "op T handles hold no copy of B");
    if (p->k * p->n == 0) return TSMM_SUCCESS;
    if (!B_out) return fail(TSMM_ERROR_INVALID_VALUE, "B_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const char *base = static_cast<const char *>(p->dev);
    hipError_t e;
    if (p->mode != TSMM_MODE_NATIVE)
        e = launch_unpack_split(base + p->L.off_planes, reinterpret_cast<const int32_t *>(base + p->L.off_exps),
                                B_out, p->k, p->n, p->L.terms, s);
    else
        e = hipMemcpyAsync(B_out, base + p->L.off_rowmajor, (size_t)p->k * p->n * elem_bytes(p->dtype),
                           hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? TSMM_SUCCESS : hip_fail(e, "unpack");
}

tsmm_status tsmm_packed_split_planes(tsmm_packed_t p, void *planes_out, void *exps_out, void *stream) {
    g_err.clear();
    if (!p) return fail(TSMM_ERROR_INVALID_VALUE, "packed is NULL");
    if (p->is_a || p->mode == TSMM_MODE_NATIVE)
        return fail(TSMM_ERROR_NOT_SUPPORTED, "not a split-mode packed B handle");
    if (p->k * p->n == 0) return TSMM_SUCCESS;
    if (!planes_out || !exps_out) return fail(TSMM_ERROR_INVALID_VALUE, "NULL output");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const char *base = static_cast<const char *>(p->dev);
    hipError_t e = hipMemcpyAsync(planes_out, base + p->L.off_planes, (size_t)p->L.terms * p->k * p->n * 2,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(exps_out, base + p->L.off_exps, (size_t)p->n * 4, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? TSMM_SUCCESS : hip_fail(e, "split planes");
}

void tsmm_packed_destroy(tsmm_packed_t p) {
    if (!p) return;
    if (p->dev) (void)hipFree(p->dev);
    delete p;
}

tsmm_status tsmm_pack_a(const void *A, int64_t m, int64_t k, int64_t lda, tsmm_dtype dtype, tsmm_mode mode,
                        double alpha, void *stream, tsmm_packed_t *out) {
    g_err.clear();
    if (!out) return fail(TSMM_ERROR_INVALID_VALUE, "out is NULL");
    *out = nullptr;
    if (m < 0 || k < 0) return fail(TSMM_ERROR_INVALID_VALUE, "negative size");
    if (!valid_dtype(dtype)) return fail(TSMM_ERROR_INVALID_VALUE, "bad dtype %d", (int)dtype);
    if (!valid_mode(mode)) return fail(TSMM_ERROR_INVALID_VALUE, "bad mode %d", (int)mode);
    if (dtype == TSMM_BF16) return fail(TSMM_ERROR_NOT_SUPPORTED, "bfloat16 A is read as it is; nothing to pack");
    if (mode != TSMM_MODE_NATIVE && dtype != TSMM_F32)
        return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes take binary32 operands");
    if (mode != TSMM_MODE_NATIVE && k > kMaxKC)
        return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes need k <= %d", kMaxKC);
    if (m > INT32_MAX * (int64_t)16 || k > INT32_MAX) return fail(TSMM_ERROR_NOT_SUPPORTED, "A too large");
    if (lda < std::max<int64_t>(1, k)) return fail(TSMM_ERROR_INVALID_VALUE, "lda %" PRId64 " < k", lda);
    if (m * k > 0 && !A) return fail(TSMM_ERROR_INVALID_VALUE, "A is NULL");

    std::unique_ptr<tsmm_packed_s> P(new (std::nothrow) tsmm_packed_s());
    if (!P) return fail(TSMM_ERROR_OUT_OF_MEMORY, "host allocation failed");
    P->is_a = true;
    P->m = m;
    P->k = k;
    P->n = 0;
    P->layout = TSMM_OP_N;
    P->dtype = dtype;
    P->mode = mode;
    P->alpha = alpha;
    const int terms = mode == TSMM_MODE_NATIVE ? 0 : split_terms(dtype, mode);
    P->L.terms = terms;
    if (m == 0 || k == 0) {  // nothing to hold
        *out = P.release();
        return TSMM_SUCCESS;
    }
    P->L.bytes = terms > 0 ? (size_t)terms * presplit_rows(m) * presplit_ld(k) * 2 : (size_t)m * k * elem_bytes(dtype);
    if (terms > 0 && k % 8 == 0) {
        // the wide kernels split A in the shadow of their products: for a plan
        // that runs them, RN32(alpha*A) itself is the cheaper operand to read
        P->L.has_a32 = true;
        P->L.off_a32 = (P->L.bytes + 255) & ~(size_t)255;
        P->L.bytes = P->L.off_a32 + (size_t)m * k * 4;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(TSMM_ERROR_NO_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    P->device = dev;
    e = dev_malloc(&P->dev, P->L.bytes, "pack_a");
    if (e != hipSuccess)
        return fail(TSMM_ERROR_OUT_OF_MEMORY, "hipMalloc(%zu): %s", P->L.bytes, hipGetErrorString(e));
    e = launch_pack_a(dtype, terms, A, lda, P->dev, m, k, alpha, static_cast<hipStream_t>(stream));
    if (e == hipSuccess && P->L.has_a32)
        e = launch_pack_a(dtype, 0, A, lda, static_cast<char *>(P->dev) + P->L.off_a32, m, k, alpha,
                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        (void)hipFree(P->dev);
        return hip_fail(e, "pack A");
    }
    *out = P.release();
    return TSMM_SUCCESS;
}

// ------------------------------------------------------------------ plan

tsmm_status tsmm_plan(int64_t m, int64_t n, int64_t k, tsmm_layout layout, tsmm_dtype dtype,
                      tsmm_plan_t *out) {
    g_err.clear();
    tsmm_status st = check_plan_args(m, n, k, layout, dtype, out);
    if (st != TSMM_SUCCESS) return st;
    *out = nullptr;
    tsmm_device_caps caps;
    int dev = 0;
    st = query_caps(&caps, &dev);
    if (st != TSMM_SUCCESS) return st;
    return make_plan(m, n, k, layout, dtype, &caps, dev, out);
}

tsmm_status tsmm_plan_with_caps(int64_t m, int64_t n, int64_t k, tsmm_layout layout, tsmm_dtype dtype,
                                const tsmm_device_caps *caps, tsmm_plan_t *out) {
    g_err.clear();
    tsmm_status st = check_plan_args(m, n, k, layout, dtype, out);
    if (st != TSMM_SUCCESS) return st;
    *out = nullptr;
    if (!caps || caps->compute_units < 1 || caps->lds_bytes_per_cu < 1)
        return fail(TSMM_ERROR_INVALID_VALUE, "bad device caps");
    return make_plan(m, n, k, layout, dtype, caps, -1, out);
}

tsmm_status tsmm_plan_set_mode(tsmm_plan_t p, tsmm_mode mode) {
    g_err.clear();
    if (!p) return fail(TSMM_ERROR_INVALID_VALUE, "plan is NULL");
    if (!valid_mode(mode)) return fail(TSMM_ERROR_INVALID_VALUE, "bad mode %d", (int)mode);
    if (p->batched) return fail(TSMM_ERROR_NOT_SUPPORTED, "batched plans run NATIVE only");
    if (mode != TSMM_MODE_NATIVE && (p->dtype != TSMM_F32 || p->layout != TSMM_OP_N))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes take op N binary32 operands");
    if (mode != TSMM_MODE_NATIVE && (!kclass32(p->k) || !ntclass(p->n)))
        return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes need k <= %d and n <= 256", kMaxKC);
    tsmm_plan_s trial = *p;
    trial.mode = mode;
    trial.workspace = nullptr;
    trial.owns_workspace = false;
    tsmm_status st = choose_tile(trial);
    if (st != TSMM_SUCCESS) return st;
    p->mode = mode;
    p->tile = trial.tile;
    p->tile_from_table = trial.tile_from_table;
    p->KC = trial.KC;
    p->NT = trial.NT;
    p->vec = trial.vec;
    p->grid = trial.grid;
    p->grid_y = trial.grid_y;
    p->block = trial.block;
    p->workspace_bytes = trial.workspace_bytes;
    return TSMM_SUCCESS;
}

tsmm_status tsmm_plan_set_tile(tsmm_plan_t p, const tsmm_tile *tile) {
    g_err.clear();
    if (!p || !tile) return fail(TSMM_ERROR_INVALID_VALUE, "NULL argument");
    if (p->batched) return set_batched_tile(*p, *tile);
    if (tile->kernel < 0 || tile->kernel > TSMM_KERNEL_COLMAJOR || tile->kernel == TSMM_KERNEL_BATCHED)
        return fail(TSMM_ERROR_INVALID_VALUE, "bad kernel id %d", tile->kernel);
    if (tile->chunk_rows != 0) return fail(TSMM_ERROR_INVALID_VALUE, "chunk_rows is for batched plans");
    tsmm_plan_s trial = *p;
    trial.workspace = nullptr;
    trial.owns_workspace = false;
    tsmm_status st = apply_tile(trial, *tile);
    if (st != TSMM_SUCCESS) return st;
    const size_t old_ws = p->workspace_bytes;
    p->tile = trial.tile;
    p->tile_from_table = false;
    p->KC = trial.KC;
    p->NT = trial.NT;
    p->vec = trial.vec;
    p->grid = trial.grid;
    p->grid_y = trial.grid_y;
    p->block = trial.block;
    p->workspace_bytes = trial.workspace_bytes;
    if (p->workspace_bytes > old_ws && p->owns_workspace) {  // grow lazily on next execute
        (void)hipFree(p->workspace);
        p->workspace = nullptr;
        p->workspace_size = 0;
        p->owns_workspace = false;
    }
    return TSMM_SUCCESS;
}

tsmm_status tsmm_plan_get_tile(tsmm_plan_t p, tsmm_tile *tile) {
    g_err.clear();
    if (!p || !tile) return fail(TSMM_ERROR_INVALID_VALUE, "NULL argument");
    *tile = p->tile;
    return TSMM_SUCCESS;
}

tsmm_status tsmm_plan_set_stream(tsmm_plan_t p, void *stream) {
    g_err.clear();
    if (!p) return fail(TSMM_ERROR_INVALID_VALUE, "plan is NULL");
    p->stream = static_cast<hipStream_t>(stream);
    return TSMM_SUCCESS;
}

tsmm_status tsmm_plan_workspace_bytes(tsmm_plan_t p, size_t *bytes) {
    g_err.clear();
    if (!p || !bytes) return fail(TSMM_ERROR_INVALID_VALUE, "NULL argument");
    *bytes = p->workspace_bytes;
    return TSMM_SUCCESS;
}

tsmm_status tsmm_plan_set_workspace(tsmm_plan_t p, void *ws, size_t bytes) {
    g_err.clear();
    if (!p) return fail(TSMM_ERROR_INVALID_VALUE, "plan is NULL");
    if (ws && bytes < p->workspace_bytes)
        return fail(TSMM_ERROR_INVALID_VALUE, "workspace of %zu bytes, the plan needs %zu", bytes, p->workspace_bytes);
    if (p->owns_workspace && p->workspace) (void)hipFree(p->workspace);
    p->workspace = ws;
    p->workspace_size = ws ? bytes : 0;
    p->owns_workspace = false;
    return TSMM_SUCCESS;
}

tsmm_status tsmm_plan_describe(tsmm_plan_t p, char *buf, size_t len) {
    g_err.clear();
    if (!p || !buf || len == 0) return fail(TSMM_ERROR_INVALID_VALUE, "NULL argument");
    snprintf(buf, len,
             "op=%c dtype=%s mode=%s m=%" PRId64 " n=%" PRId64 " k=%" PRId64
             " kernel=%s kc=%d nt=%d vec=%d rt=%d waves=%d wg_per_cu=%d splitk=%d nsplit=%d grid=%" PRId64 "x%" PRId64
             " block=%d workspace=%zu table=%d ran=%s",
             p->layout == TSMM_OP_N ? 'N' : (p->layout == TSMM_OP_T ? 'T' : 'C'), dtype_name(p->dtype), mode_name(p->mode), p->m, p->n, p->k,
             kernel_name(p->tile.kernel), p->KC, p->NT, (int)p->vec, p->tile.rows_per_wave, p->tile.waves_per_wg,
             p->tile.wg_per_cu, p->tile.splitk, p->tile.nsplit, p->grid, p->grid_y, p->block, p->workspace_bytes,
             (int)p->tile_from_table, p->last_kernel ? kernel_name(p->last_kernel) : "-");
    return TSMM_SUCCESS;
}

void tsmm_plan_destroy(tsmm_plan_t p) {
    if (!p) return;
    if (p->owns_workspace && p->workspace) (void)hipFree(p->workspace);
    if (p->d_desc) (void)hipFree(p->d_desc);
    if (p->d_inst_start) (void)hipFree(p->d_inst_start);
    if (p->d_ctr) (void)hipFree(p->d_ctr);
    if (p->h_desc) (void)hipHostFree(p->h_desc);
    delete p;
}

// --------------------------------------------------------------- execute

}  // extern "C"

namespace {
// The plan's device scratch: the caller's (tsmm_plan_set_workspace), else
// allocated on first use and owned by the plan.
tsmm_status ensure_workspace(tsmm_plan_s &p) {
    if (p.workspace_bytes == 0 || (p.workspace && p.workspace_size >= p.workspace_bytes)) return TSMM_SUCCESS;
    if (p.owns_workspace && p.workspace) (void)hipFree(p.workspace);
    p.workspace = nullptr;
    p.owns_workspace = false;
    void *ws = nullptr;
    hipError_t e = dev_malloc(&ws, p.workspace_bytes, "workspace");
    if (e != hipSuccess)
        return fail(TSMM_ERROR_OUT_OF_MEMORY, "workspace (%zu bytes): %s", p.workspace_bytes, hipGetErrorString(e));
    p.workspace = ws;
    p.workspace_size = p.workspace_bytes;
    p.owns_workspace = true;
    return TSMM_SUCCESS;
}
}  // namespace

extern "C" {

// Natural strides of a plan's operands: A's and C's row stride (op N,
// op T) or column stride (column-major).
// Natural strides (at least 1, as in BLAS, also for empty matrices).
void natural_ld(const tsmm_plan_s &p, int64_t *lda, int64_t *ldc) {
    if (p.layout == TSMM_OP_N) {
        *lda = p.k;
        *ldc = p.n;
    } else if (p.layout == TSMM_OP_T) {
        *lda = p.m;
        *ldc = p.n;
    } else {
        *lda = p.m;
        *ldc = p.m;
    }
    *lda = std::max<int64_t>(1, *lda);
    *ldc = std::max<int64_t>(1, *ldc);
}

tsmm_status tsmm_execute(tsmm_plan_t p, const void *A, tsmm_packed_t packed, void *C, double alpha,
                         double beta) {
    if (!p) {
        g_err.clear();
        return fail(TSMM_ERROR_INVALID_VALUE, "NULL plan or packed operand");
    }
    int64_t lda, ldc;
    natural_ld(*p, &lda, &ldc);
    return tsmm_execute_ld(p, A, lda, packed, C, ldc, alpha, beta);
}

}  // extern "C"

namespace {
// tsmm_execute_ld with the split-k partial sums in `scratch` (at least the
// plan's workspace bytes) when it is not NULL, else in the plan's
// workspace (the caller's, or allocated on first use).
tsmm_status execute_core(tsmm_plan_t p, const void *A, int64_t lda, tsmm_packed_t packed, void *C, int64_t ldc,
                         double alpha, double beta, void *scratch) {
    if (!p || !packed) return fail(TSMM_ERROR_INVALID_VALUE, "NULL plan or packed operand");
    if (p->batched) return fail(TSMM_ERROR_INVALID_VALUE, "batched plan: use tsmm_execute_batched");
    if (p->device < 0) return fail(TSMM_ERROR_NO_DEVICE, "plan was built for explicit caps, not a device");
    if (packed->is_a) return fail(TSMM_ERROR_INVALID_VALUE, "a packed A handle was passed as the packed B operand");
    if (packed->k != p->k || packed->n != p->n || packed->dtype != p->dtype || packed->layout != p->layout ||
        packed->mode != p->mode)
        return fail(TSMM_ERROR_SHAPE_MISMATCH,
                    "plan (k=%" PRId64 " n=%" PRId64 " %s %s) vs packed (k=%" PRId64 " n=%" PRId64 " %s %s)", p->k,
                    p->n, dtype_name(p->dtype), mode_name(p->mode), packed->k, packed->n,
                    dtype_name(packed->dtype), mode_name(packed->mode));
    int64_t nat_a, nat_c;
    natural_ld(*p, &nat_a, &nat_c);
    if (lda < nat_a || ldc < nat_c)
        return fail(TSMM_ERROR_INVALID_VALUE, "lda %" PRId64 " / ldc %" PRId64 " below the natural %" PRId64
                                              " / %" PRId64, lda, ldc, nat_a, nat_c);
    if (p->m == 0 || p->n == 0) return TSMM_SUCCESS;
    if (!C) return fail(TSMM_ERROR_INVALID_VALUE, "C is NULL");
    if (alpha != 0.0 && p->k > 0 && !A) return fail(TSMM_ERROR_INVALID_VALUE, "A is NULL");
    const bool strided = lda != nat_a || ldc != nat_c;
    const tsmm_dtype out_dt = p->dtype == TSMM_F64 ? TSMM_F64 : TSMM_F32;
    hipStream_t s = p->stream;
    const char *base = static_cast<const char *>(packed->dev);
    // the caller's copy of B: row-major (op N), column-major (TSMM_COLMAJOR)
    const void *Brow = p->layout != TSMM_OP_T ? base + packed->L.off_rowmajor : nullptr;
    // the any-shape kernel, with strides (column-major: row-major C^T = B^T A^T)
    auto simple = [&](double a, int64_t kk) -> hipError_t {
        if (p->layout == TSMM_OP_T)
            return launch_simple_ld(p->dtype, true, A, lda, packed->ref, p->n, C, ldc, p->m, p->n, kk, a, beta, s);
        if (p->layout == TSMM_COLMAJOR)
            return launch_simple_ld(p->dtype, false, Brow, p->k, A, lda, C, ldc, p->n, p->m, kk, a, beta, s);
        return launch_simple_ld(p->dtype, false, A, lda, Brow, p->n, C, ldc, p->m, p->n, kk, a, beta, s);
    };
    hipError_t e;
    if (alpha == 0.0 || p->k == 0) {
        if (strided) {  // C = beta*C through the strided any-shape kernel (no product terms)
            e = simple(0.0, 0);
        } else {
            e = launch_scale(out_dt, C, p->m * p->n, beta, s);
        }
        return e == hipSuccess ? TSMM_SUCCESS : hip_fail(e, "scale launch");
    }
    const int vw = 16 / elem_bytes(p->dtype);
    const bool a16 = (reinterpret_cast<uintptr_t>(A) & 15) == 0, c16 = (reinterpret_cast<uintptr_t>(C) & 15) == 0;
    // strides the 32-bit lane offsets of the row-major kernels cover
    // strides the row-major kernels' tile resources cover: 16 rows of
    // either operand span at most 2^30 bytes, so the out-of-range offset
    // kOOB (2^30) lies past every tile and the lane offsets fit 32 bits
    const int64_t eb_in = elem_bytes(p->dtype), eb_out = elem_bytes(out_dt);
    const bool ld32 = lda * eb_in <= ((int64_t)1 << 26) && ldc * eb_out <= ((int64_t)1 << 26);
    int kernel = p->tile.kernel;
    if (kernel == TSMM_KERNEL_STREAM || kernel == TSMM_KERNEL_SLAB) {
        const bool il = frag4_pg(p->dtype, p->NT, p->n) > 1;
        if (!ld32 || (p->vec && (!a16 || lda % vw)) || (il && (!c16 || ldc % vw)))
            kernel = TSMM_KERNEL_SIMPLE;  // vector accesses need 16-byte aligned rows
    } else if (kernel == TSMM_KERNEL_COLMAJOR) {
        if (!a16 || !c16 || lda % vw || ldc % vw) kernel = TSMM_KERNEL_SIMPLE;
    } else if (kernel == TSMM_KERNEL_SPLITK || kernel == TSMM_KERNEL_VALU64) {
        if (strided || (kernel == TSMM_KERNEL_VALU64 && (!a16 || !c16))) kernel = TSMM_KERNEL_SIMPLE;
    } else if (kernel == TSMM_KERNEL_SPLITBF16 || kernel == TSMM_KERNEL_WIDE) {
        const bool il = kernel == TSMM_KERNEL_WIDE || bfrag_pg(p->dtype, p->NT, p->n) > 1;
        const bool needs_c16 = il;
        if (strided || !a16 || (needs_c16 && !c16)) {
            if (p->mode != TSMM_MODE_NATIVE)
                return fail(TSMM_ERROR_INVALID_VALUE,
                            "split-bf16 modes need natural strides and 16-byte aligned A (and C)");
            kernel = TSMM_KERNEL_SIMPLE;
        }
    }
    if (kernel != p->tile.kernel && p->last_kernel != kernel && log_level() >= 1) {
        char buf[256];
        tsmm_plan_describe(p, buf, sizeof buf);
        fprintf(stderr, "[tsmm] execute runs the %s kernel instead of the plan's (operand alignment or strides): %s\n",
                kernel_name(kernel), buf);
    }
    p->last_kernel = kernel;
    switch (kernel) {
    case TSMM_KERNEL_STREAM: {
        // C in 16-byte vectors: interleaved columns where the fragments
        // have them, else (binary64, one column tile, n even) lane pairs
        // when C and ldc allow it, else element by element
        int cm = frag4_pg(p->dtype, p->NT, p->n) > 1 ? 1 : 0;
        if (cm == 0 && p->dtype == TSMM_F64 && p->NT == 1 && p->n % 2 == 0 && c16 && ldc % 2 == 0 &&
            stream_variant_exists(p->dtype, p->KC, 1, p->tile.rows_per_wave, p->vec, 2))
            cm = 2;
        // beta == 0 on the memory-bound binary64 classes: default-policy C
        // stores (measured faster there; streaming stores where C is read)
        if (cm != 0 && beta == 0.0 && p->dtype == TSMM_F64 && p->KC <= 64 &&
            stream_variant_exists(p->dtype, p->KC, p->NT / p->tile.nsplit, p->tile.rows_per_wave, p->vec, cm | 4))
            cm |= 4;
        e = launch_stream(p->dtype, p->KC, p->NT / p->tile.nsplit, p->tile.rows_per_wave, p->vec, cm, A,
                          base + packed->L.off_frag, C, p->m, p->n, p->k, lda, ldc, alpha, beta, p->grid, p->block,
                          p->NT, p->tile.nsplit, s);
        break;
    }
    case TSMM_KERNEL_VALU64:
        e = launch_valu64(p->tile.rows_per_wave, static_cast<const double *>(A), static_cast<const double *>(Brow),
                          static_cast<double *>(C), p->m, p->n, p->k, alpha, beta, p->grid, s);
        break;
    case TSMM_KERNEL_SPLITBF16: {
        const bool il = bfrag_pg(p->dtype, p->NT, p->n) > 1;
        e = launch_splitbf16(p->dtype, p->KC, p->NT / p->tile.nsplit, p->tile.rows_per_wave,
                             split_products(p->dtype, p->mode), il, A, base + packed->L.off_frag,
                             p->mode != TSMM_MODE_NATIVE ? reinterpret_cast<const int32_t *>(base + packed->L.off_exps)
                                                         : nullptr,
                             C, p->m, p->n, p->k, alpha, beta, p->grid, p->block, p->NT, p->tile.nsplit, s);
        break;
    }
    case TSMM_KERNEL_WIDE:
        if (!packed->L.wide_KC || packed->L.wide_KC != p->KC)
            return fail(TSMM_ERROR_SHAPE_MISMATCH, "packed operand has no image for the wide kernel");
        e = launch_wide(wide_products(*p), p->KC, p->NT, p->tile.rows_per_wave, p->tile.waves_per_wg, A,
                        base + packed->L.off_wide,
                        p->mode != TSMM_MODE_NATIVE ? reinterpret_cast<const int32_t *>(base + packed->L.off_exps)
                                                    : nullptr,
                        C, p->m, p->n, p->k, alpha, beta, p->grid, s);
        break;
    case TSMM_KERNEL_COLMAJOR:
        e = launch_colmajor(p->dtype, p->KC, p->NT / (p->tile.nsplit * p->tile.rows_per_wave), p->tile.rows_per_wave,
                            A, base + packed->L.off_frag, C, p->m, p->n, p->k, lda, ldc, alpha, beta, p->grid, p->NT,
                            p->tile.nsplit, s);
        break;
    case TSMM_KERNEL_SLAB: {
        const bool il = frag4_pg(p->dtype, p->NT, p->n) > 1;
        if (packed->L.KC != p->KC || packed->L.NT != p->NT)
            return fail(TSMM_ERROR_SHAPE_MISMATCH, "packed operand has no image for the k-slab kernel");
        tsmm_status st = scratch ? TSMM_SUCCESS : ensure_workspace(*p);
        if (st != TSMM_SUCCESS) return st;
        e = launch_slab(p->dtype, p->NT, p->tile.rows_per_wave, p->vec, il, A, base + packed->L.off_frag, C,
                        static_cast<double *>(scratch ? scratch : p->workspace), p->m, p->n, p->k, lda, ldc, p->KC,
                        alpha, beta, p->tile.splitk, p->grid, s);
        break;
    }
    case TSMM_KERNEL_SPLITK: {
        tsmm_status st = scratch ? TSMM_SUCCESS : ensure_workspace(*p);
        if (st != TSMM_SUCCESS) return st;
        e = launch_splitk(p->KC, p->NT, p->tile.rows_per_wave, static_cast<const double *>(A),
                          static_cast<const double *>(packed->ref),
                          static_cast<double *>(scratch ? scratch : p->workspace), static_cast<double *>(C), p->k,
                          p->m, p->n, p->tile.splitk, alpha, beta, p->block, s);
        break;
    }
    default:
        e = simple(alpha, p->k);
        break;
    }
    return e == hipSuccess ? TSMM_SUCCESS : hip_fail(e, "kernel launch");
}
}  // namespace

extern "C" {

tsmm_status tsmm_execute_ld(tsmm_plan_t p, const void *A, int64_t lda, tsmm_packed_t packed, void *C, int64_t ldc,
                            double alpha, double beta) {
    g_err.clear();
    return execute_core(p, A, lda, packed, C, ldc, alpha, beta, nullptr);
}

tsmm_status tsmm_execute_noalloc(tsmm_plan_t p, const void *A, tsmm_packed_t packed, void *C, double alpha,
                                 double beta) {
    g_err.clear();
    if (!p || !packed) return fail(TSMM_ERROR_INVALID_VALUE, "NULL plan or packed operand");
    if (p->batched) return fail(TSMM_ERROR_INVALID_VALUE, "batched plan: use tsmm_execute_batched");
    if (p->device < 0) return fail(TSMM_ERROR_NO_DEVICE, "plan was built for explicit caps, not a device");
    if (p->workspace_bytes > kScratchBytes)
        return fail(TSMM_ERROR_NOT_SUPPORTED,
                    "the plan needs %zu bytes of scratch; the static scratch holds %zu (fewer split-k parts, or "
                    "tsmm_execute with a workspace)",
                    p->workspace_bytes, kScratchBytes);
    int64_t nat_a, nat_c;
    natural_ld(*p, &nat_a, &nat_c);
    void *scratch = nullptr;
    if (p->workspace_bytes > 0 && p->m > 0 && p->n > 0 && p->k > 0 && alpha != 0.0) {
        const hipError_t e = scratch_device_ptr(p->device, &scratch);
        if (e != hipSuccess) return hip_fail(e, "static scratch address");
    }
    return execute_core(p, A, nat_a, packed, C, nat_c, alpha, beta, scratch);
}

// ------------------------------------------------------ runtime evaluator

}  // extern "C"

namespace {
// Candidate tiles of the plan's kernel family (the paper's two search
// patterns over the register / thread blocking: multiples of the tile under
// the capacity bounds, and powers of two), the plan's current tile first.
std::vector<tsmm_tile> tune_candidates(const tsmm_plan_s &p) {
    std::vector<tsmm_tile> out;
    out.push_back(p.tile);
    auto add = [&](int kernel, int rt, int wpc, int sk, int ns) {
        out.push_back(tsmm_tile{kernel, rt, 4, wpc, sk, ns, 0});
    };
    const int nat = natural_kernel(p);
    const tsmm_tile d = default_tile(p, nat);
    switch (nat) {
    case TSMM_KERNEL_STREAM:
        for (int ns : {d.nsplit, 2 * d.nsplit})
            for (int rt : {1, 2, 4, 8})
                for (int wpc : {1, 2, 4, 8, 16}) add(nat, rt, wpc, 1, ns);
        break;
    case TSMM_KERNEL_SPLITBF16:
        for (int ns : {d.nsplit, 2 * d.nsplit})
            for (int rt : {1, 2})
                for (int wpc : {1, 2, 4, 8}) add(nat, rt, wpc, 1, ns);
        break;
    case TSMM_KERNEL_SPLITK:
        for (int rg : {1, 2, 4})
            for (int P : {256, 512, 1024, 2048}) add(nat, rg, 1, P, 1);
        break;
    case TSMM_KERNEL_SLAB:
        for (int rt : {1, 2, 4})
            for (int sk : {1, 2, 3, 4, 5, 6, 8, 12, 16}) add(nat, rt, 1, sk, 1);
        break;
    case TSMM_KERNEL_COLMAJOR:
        for (int ng : {1, 2})
            for (int ns : {d.nsplit * d.rows_per_wave / ng, 2 * d.nsplit * d.rows_per_wave / ng})
                for (int wpc : {1, 2, 4, 8, 16})
                    if (ns >= 1) add(nat, ng, wpc, 1, ns);
        break;
    default:
        break;
    }
    if (wide_ok(p)) {
        for (int rt : {2, 4}) add(TSMM_KERNEL_WIDE, rt, 1, 1, 1);
        out.push_back(tsmm_tile{TSMM_KERNEL_WIDE, 1, 8, 1, 1, 1, 0});  // two wavefronts per SIMD
    }
    return out;
}
}  // namespace

extern "C" {

// The split-bf16 geometry that runs a pre-split A for plan p: the plan's
// own tile when it runs the split-bf16 kernel, else that kernel's default;
// rows per wavefront halve, then column groups double, until a pre-split
// variant exists.
static tsmm_status presplit_geometry(const tsmm_plan_s &p, tsmm_plan_s &q) {
    const int KC = kclass32(p.k), NT = ntclass(p.n), prod = split_products(p.dtype, p.mode);
    if (!KC || !NT) return fail(TSMM_ERROR_NOT_SUPPORTED, "split-bf16 modes need k <= %d and n <= 256", kMaxKC);
    const int pg = bfrag_pg(p.dtype, NT, p.n);  // the packed B's column interleave group
    tsmm_tile t = p.tile.kernel == TSMM_KERNEL_SPLITBF16 ? p.tile : default_tile(p, TSMM_KERNEL_SPLITBF16);
    t.kernel = TSMM_KERNEL_SPLITBF16;
    t.nsplit = std::max(1, std::min(t.nsplit, NT / pg));
    for (;;) {
        const int NTs = NT / t.nsplit;
        int rt = std::max(1, t.rows_per_wave);
        while (rt > 1 && !splitbf16_presplit_exists(prod, KC, NTs, rt, pg > 1)) rt /= 2;
        if (splitbf16_presplit_exists(prod, KC, NTs, rt, pg > 1)) {
            t.rows_per_wave = rt;
            break;
        }
        if (t.nsplit * 2 > NT / pg)
            return fail(TSMM_ERROR_NOT_SUPPORTED, "no pre-split kernel for KC=%d NT=%d", KC, NT);
        t.nsplit *= 2;
    }
    q = p;
    q.workspace = nullptr;
    q.owns_workspace = false;
    return apply_tile(q, t);
}

tsmm_status tsmm_execute_packed_a(tsmm_plan_t p, tsmm_packed_t packed_a, tsmm_packed_t packed, void *C,
                                  double beta) {
    g_err.clear();
    if (!p || !packed_a || !packed) return fail(TSMM_ERROR_INVALID_VALUE, "NULL plan or packed operand");
    if (!packed_a->is_a) return fail(TSMM_ERROR_INVALID_VALUE, "packed_a is not a packed A handle");
    if (p->batched) return fail(TSMM_ERROR_INVALID_VALUE, "batched plan: use tsmm_execute_batched");
    if (p->layout != TSMM_OP_N) return fail(TSMM_ERROR_NOT_SUPPORTED, "packed A serves op N plans");
    if (packed_a->m != p->m || packed_a->k != p->k || packed_a->dtype != p->dtype || packed_a->mode != p->mode)
        return fail(TSMM_ERROR_SHAPE_MISMATCH,
                    "plan (m=%" PRId64 " k=%" PRId64 " %s %s) vs packed A (m=%" PRId64 " k=%" PRId64 " %s %s)", p->m,
                    p->k, dtype_name(p->dtype), mode_name(p->mode), packed_a->m, packed_a->k,
                    dtype_name(packed_a->dtype), mode_name(packed_a->mode));
    // alpha = 0 at pack time: reference-BLAS convention, neither A nor B is read
    const double alpha = packed_a->alpha == 0.0 ? 0.0 : 1.0;
    if (p->mode == TSMM_MODE_NATIVE || alpha == 0.0 || p->k == 0 || p->m == 0 || p->n == 0)
        return tsmm_execute(p, packed_a->dev, packed, C, alpha, beta);
    if (packed->is_a) return fail(TSMM_ERROR_INVALID_VALUE, "a packed A handle was passed as the packed B operand");
    if (p->device < 0) return fail(TSMM_ERROR_NO_DEVICE, "plan was built for explicit caps, not a device");
    if (packed->k != p->k || packed->n != p->n || packed->dtype != p->dtype || packed->layout != p->layout ||
        packed->mode != p->mode)
        return fail(TSMM_ERROR_SHAPE_MISMATCH, "plan and packed B disagree");
    if (!C) return fail(TSMM_ERROR_INVALID_VALUE, "C is NULL");
    if (reinterpret_cast<uintptr_t>(C) & 3) return fail(TSMM_ERROR_INVALID_VALUE, "C must be 4-byte aligned");
    if (p->tile.kernel == TSMM_KERNEL_WIDE && packed_a->L.has_a32)
        // the plan's wide kernel on RN32(alpha*A): it splits each value into
        // the same terms as the pre-split planes hold
        return tsmm_execute(p, static_cast<const char *>(packed_a->dev) + packed_a->L.off_a32, packed, C, 1.0, beta);
    const bool il = packed->L.pg > 1;  // C in 16-byte vectors
    if (il && (reinterpret_cast<uintptr_t>(C) & 15))
        return fail(TSMM_ERROR_INVALID_VALUE, "C must be 16-byte aligned when n is a multiple of 4 and n > 48");
    tsmm_plan_s q;
    const tsmm_status st = presplit_geometry(*p, q);
    if (st != TSMM_SUCCESS) return st;
    const char *base = static_cast<const char *>(packed->dev);
    p->last_kernel = TSMM_KERNEL_SPLITBF16;
    const hipError_t e = launch_splitbf16_presplit(
        split_products(p->dtype, p->mode), q.KC, q.NT / q.tile.nsplit, q.tile.rows_per_wave, il, packed_a->dev,
        base + packed->L.off_frag, reinterpret_cast<const int32_t *>(base + packed->L.off_exps), C, p->m, p->n, p->k,
        beta, q.grid, q.block, q.NT, q.tile.nsplit, p->stream);
    return e == hipSuccess ? TSMM_SUCCESS : hip_fail(e, "pre-split launch");
}

tsmm_status tsmm_plan_tune(tsmm_plan_t p, const void *A, tsmm_packed_t packed, void *C, int reps, double *best_ms) {
    g_err.clear();
    if (!p || !packed || !C) return fail(TSMM_ERROR_INVALID_VALUE, "NULL plan, packed operand or C");
    if (p->batched) return fail(TSMM_ERROR_INVALID_VALUE, "batched plans take their tile with tsmm_plan_set_tile");
    if (p->device < 0) return fail(TSMM_ERROR_NO_DEVICE, "plan was built for explicit caps, not a device");
    if (reps < 1 || reps > 1000) return fail(TSMM_ERROR_INVALID_VALUE, "reps must be in 1..1000");
    if (best_ms) *best_ms = 0.0;
    if (p->m == 0 || p->n == 0 || p->k == 0) return TSMM_SUCCESS;  // nothing runs
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "evaluator events");
    }
    const tsmm_tile orig = p->tile;
    const int orig_src = p->tile_from_table;
    double best = -1.0;
    tsmm_tile best_tile = orig;
    tsmm_status st = TSMM_SUCCESS;
    for (const tsmm_tile &cand : tune_candidates(*p)) {
        if (tsmm_plan_set_tile(p, &cand) != TSMM_SUCCESS) continue;  // not for this shape or device
        st = tsmm_execute(p, A, packed, C, 1.0, 0.0);  // warm-up
        if (st != TSMM_SUCCESS) break;
        std::vector<float> ms;
        for (int r = 0; r < reps && st == TSMM_SUCCESS; ++r) {
            e = hipEventRecord(e0, p->stream);
            if (e == hipSuccess) st = tsmm_execute(p, A, packed, C, 1.0, 0.0);
            if (e == hipSuccess && st == TSMM_SUCCESS) e = hipEventRecord(e1, p->stream);
            if (e == hipSuccess && st == TSMM_SUCCESS) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess && st == TSMM_SUCCESS) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess && st == TSMM_SUCCESS) st = hip_fail(e, "evaluator timing");
            ms.push_back(t);
        }
        if (st != TSMM_SUCCESS) break;
        std::sort(ms.begin(), ms.end());
        const double med = ms[ms.size() / 2];
        if (best < 0.0 || med < best) {
            best = med;
            best_tile = p->tile;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != TSMM_SUCCESS || best < 0.0) {
        const std::string err = g_err;
        (void)tsmm_plan_set_tile(p, &orig);
        p->tile_from_table = orig_src;
        g_err = err;
        return st != TSMM_SUCCESS ? st : fail(TSMM_ERROR_NOT_SUPPORTED, "no candidate tile runs this plan");
    }
    st = tsmm_plan_set_tile(p, &best_tile);
    if (st != TSMM_SUCCESS) return st;
    p->tile_from_table = 2;
    {
        RuntimeCache &rc = runtime_cache();
        std::lock_guard<std::mutex> lock(rc.mu);
        rc.entries[plan_key(*p)] = p->tile;
    }
    if (best_ms) *best_ms = best;
    return TSMM_SUCCESS;
}

void tsmm_tune_cache_clear(void) {
    RuntimeCache &rc = runtime_cache();
    std::lock_guard<std::mutex> lock(rc.mu);
    rc.entries.clear();
}

// --------------------------------------------------------------- batched

tsmm_status tsmm_plan_batched(int64_t count, const int64_t *m, const int64_t *n, const int64_t *k,
                              tsmm_dtype dtype, tsmm_plan_t *out) {
    g_err.clear();
    if (!out) return fail(TSMM_ERROR_INVALID_VALUE, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > (1 << 24)) return fail(TSMM_ERROR_INVALID_VALUE, "count must be in 1..2^24");
    if (!m || !n || !k) return fail(TSMM_ERROR_INVALID_VALUE, "NULL shape array");
    if (dtype != TSMM_F32 && dtype != TSMM_BF16)
        return fail(TSMM_ERROR_NOT_SUPPORTED, "batched plans take TSMM_F32 or TSMM_BF16");
    for (int64_t b = 0; b < count; ++b) {
        if (m[b] < 0 || m[b] > (INT64_C(1) << 40))
            return fail(TSMM_ERROR_INVALID_VALUE, "instance %" PRId64 ": bad m", b);
        if (k[b] < 1 || k[b] > 128 || n[b] < 1 || n[b] > 128)
            return fail(TSMM_ERROR_NOT_SUPPORTED, "instance %" PRId64 ": batched k and n must be in 1..128", b);
    }
    tsmm_device_caps caps;
    int dev = 0;
    tsmm_status st = query_caps(&caps, &dev);
    if (st != TSMM_SUCCESS) return st;

    std::unique_ptr<tsmm_plan_s> p(new (std::nothrow) tsmm_plan_s());
    if (!p) return fail(TSMM_ERROR_OUT_OF_MEMORY, "host allocation failed");
    p->batched = true;
    p->dtype = dtype;
    p->layout = TSMM_OP_N;
    p->caps = caps;
    p->device = dev;
    p->inst.resize(count);
    const int sa = elem_bytes(dtype);
    std::vector<double> cost(count);
    for (int64_t b = 0; b < count; ++b) {
        p->inst[b] = {m[b], n[b], k[b]};
        // bytes of one row (A row + C row) plus a per-tile latency term
        cost[b] = (double)m[b] * (double)(k[b] * sa + n[b] * 4);
    }
    p->order.resize(count);
    for (int64_t b = 0; b < count; ++b) p->order[b] = b;
    // instances of one kernel variant (k class, n class, k-slot mapping) next
    // to each other, longest first within a variant: the workgroups that
    // share an XCD then mostly run the same code on the same B classes
    auto variant = [&](int64_t b) {
        const int KC = dtype == TSMM_BF16 ? kclass32(k[b]) : kclass4(k[b]);
        const bool vec = dtype == TSMM_BF16 ? (k[b] % 8 == 0) : vec_mapping(dtype, k[b], KC);
        return std::make_tuple(KC, ntclass(n[b]), vec);
    };
    std::stable_sort(p->order.begin(), p->order.end(), [&](int64_t x, int64_t y) {
        const auto vx = variant(x), vy = variant(y);
        return vx != vy ? vx < vy : cost[x] > cost[y];
    });

    for (const BatchedInstance &I : p->inst) {
        const int KC = dtype == TSMM_BF16 ? kclass32(I.k) : kclass4(I.k);
        p->batch_lds = std::max(p->batch_lds, batched_lds_bytes(dtype, KC, ntclass(I.n)));
    }
    // the batched kernel's fixed workgroup (kBatchWaves wavefronts), one
    // per compute unit (two wavefronts per SIMD) unless the table asks for
    // more; chunks are handed out at run time, so the grid only needs to
    // fill the device
    bool from_table = false;
    int wpc = 1;
    const int chunk = batched_table_chunk(dtype, p->caps, &from_table, &wpc);
    if (!batched_wpc_fits(*p, wpc)) wpc = 1;
    p->tile = tsmm_tile{TSMM_KERNEL_BATCHED, 0, kBatchWaves, wpc, 1, 1, chunk};
    p->tile_from_table = from_table;
    p->block = 64 * kBatchWaves;

    void *dd = nullptr, *ds = nullptr, *dc = nullptr, *hd = nullptr;
    hipError_t e1 = dev_malloc(&dd, sizeof(BatchDesc) * count, "batched");
    hipError_t e2 = dev_malloc(&ds, sizeof(int64_t) * (count + 1), "batched");
    hipError_t e3 = dev_malloc(&dc, sizeof(int32_t) * 2, "batched");
    hipError_t e5 = host_malloc_pinned(&hd, sizeof(BatchDesc) * count, "batched");
    p->d_desc = dd;
    p->d_inst_start = ds;
    p->d_ctr = dc;
    p->h_desc = hd;
    if (e1 || e2 || e3 || e5) {
        tsmm_plan_destroy(p.release());
        return fail(TSMM_ERROR_OUT_OF_MEMORY, "batched plan allocation failed");
    }
    hipError_t e = prepare_batched(dtype, p->batch_lds);
    if (e != hipSuccess) {
        tsmm_plan_destroy(p.release());
        return hip_fail(e, "batched kernel attributes");
    }
    st = batched_chunks(*p, chunk);
    if (st != TSMM_SUCCESS) {
        tsmm_plan_destroy(p.release());
        return st;
    }
    // the counters start at zero once; every launch leaves them at zero
    e = hipMemset(p->d_ctr, 0, sizeof(int32_t) * 2);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        tsmm_plan_destroy(p.release());
        return hip_fail(e, "batched plan upload");
    }
    p->m = 0;
    for (const BatchedInstance &I : p->inst) p->m += I.m;
    if (log_level() >= 1)
        fprintf(stderr, "[tsmm] batched plan: %" PRId64 " instances, %" PRId64 " chunks of %d rows, grid %" PRId64 "\n",
                count, p->n_work, chunk, p->grid);
    *out = p.release();
    return TSMM_SUCCESS;
}

tsmm_status tsmm_batched_bind(tsmm_plan_t p, const void *const *A, const tsmm_packed_t *packed, void *const *C,
                              const double *alpha, const double *beta) {
    g_err.clear();
    if (!p || !p->batched) return fail(TSMM_ERROR_INVALID_VALUE, "not a batched plan");
    if (!A || !packed || !C) return fail(TSMM_ERROR_INVALID_VALUE, "NULL operand array");
    const int64_t count = (int64_t)p->inst.size();
    std::vector<BatchDesc> desc(count);
    for (int64_t e = 0; e < count; ++e) {
        const int64_t b = p->order[e];
        const BatchedInstance &I = p->inst[b];
        const tsmm_packed_s *P = packed[b];
        if (!P) return fail(TSMM_ERROR_INVALID_VALUE, "instance %" PRId64 ": packed is NULL", b);
        if (P->is_a || P->k != I.k || P->n != I.n || P->dtype != p->dtype || P->layout != TSMM_OP_N ||
            P->mode != TSMM_MODE_NATIVE || !P->dev || !P->L.KC || !P->L.NT)
            return fail(TSMM_ERROR_SHAPE_MISMATCH, "instance %" PRId64 ": packed operand does not match", b);
        if (I.m > 0 && (!A[b] || !C[b])) return fail(TSMM_ERROR_INVALID_VALUE, "instance %" PRId64 ": NULL A or C", b);
        const bool vec = p->dtype == TSMM_BF16 ? (I.k % 8 == 0) : P->L.vec;
        if (vec && (reinterpret_cast<uintptr_t>(A[b]) & 15))
            return fail(TSMM_ERROR_INVALID_VALUE, "instance %" PRId64 ": A must be 16-byte aligned", b);
        const bool il = P->L.pg > 1;
        if (il && (reinterpret_cast<uintptr_t>(C[b]) & 15))
            return fail(TSMM_ERROR_INVALID_VALUE, "instance %" PRId64 ": C must be 16-byte aligned", b);
        BatchDesc &d = desc[e];
        memset(&d, 0, sizeof d);
        d.A = A[b];
        d.Bfrag = static_cast<const char *>(P->dev) + P->L.off_frag;
        d.C = C[b];
        d.alpha = alpha ? alpha[b] : 1.0;
        d.beta = beta ? beta[b] : 0.0;
        d.m = (d.alpha == 0.0) ? 0 : I.m;  // alpha == 0 handled below
        d.k = (int32_t)I.k;
        d.n = (int32_t)I.n;
        d.KC = P->L.KC;
        d.NT = P->L.NT;
        d.vec = vec ? 1 : 0;
        d.il = il ? 1 : 0;
        d.chunk_rows = batch_instance_chunk(p->tile.chunk_rows, I.k, I.n, (int)elem_bytes(p->dtype));
        if (d.alpha == 0.0 && I.m > 0)
            return fail(TSMM_ERROR_NOT_SUPPORTED, "instance %" PRId64 ": alpha == 0 in a batched plan", b);
    }
    if (p->bound && desc.size() == p->bound_desc.size() &&
        memcmp(desc.data(), p->bound_desc.data(), sizeof(BatchDesc) * count) == 0)
        return TSMM_SUCCESS;
    // stage through pinned memory: the copy is stream-ordered (and capturable);
    // wait for any copy still reading the staging buffer first
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "batched bind");
    memcpy(p->h_desc, desc.data(), sizeof(BatchDesc) * count);
    e = hipMemcpyAsync(p->d_desc, p->h_desc, sizeof(BatchDesc) * count, hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "batched bind");
    p->bound_desc.swap(desc);
    p->bound = true;
    return TSMM_SUCCESS;
}

tsmm_status tsmm_execute_batched(tsmm_plan_t p, const void *const *A, const tsmm_packed_t *packed, void *const *C,
                                 const double *alpha, const double *beta) {
    g_err.clear();
    if (!p || !p->batched) return fail(TSMM_ERROR_INVALID_VALUE, "not a batched plan");
    if (A) {
        tsmm_status st = tsmm_batched_bind(p, A, packed, C, alpha, beta);
        if (st != TSMM_SUCCESS) return st;
    }
    if (!p->bound) return fail(TSMM_ERROR_INVALID_VALUE, "batched plan has no bound operands");
    if (p->n_work == 0) return TSMM_SUCCESS;
    hipError_t e = launch_batched(p->dtype, static_cast<const BatchDesc *>(p->d_desc),
                                  static_cast<const int64_t *>(p->d_inst_start), p->n_work,
                                  p->tile.chunk_rows, static_cast<int32_t *>(p->d_ctr), p->grid, p->block, p->batch_lds, p->stream);
    return e == hipSuccess ? TSMM_SUCCESS : hip_fail(e, "batched launch");
}

tsmm_status tsmm_graph_create_batched(tsmm_plan_t p, tsmm_graph_t *out) {
    g_err.clear();
    if (!out) return fail(TSMM_ERROR_INVALID_VALUE, "out is NULL");
    *out = nullptr;
    if (!p || !p->batched) return fail(TSMM_ERROR_INVALID_VALUE, "not a batched plan");
    if (!p->bound) return fail(TSMM_ERROR_INVALID_VALUE, "batched plan has no bound operands");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "graph stream");
    // the descriptor upload must have landed before the graph's reads
    e = hipStreamSynchronize(p->stream);
    std::unique_ptr<tsmm_graph_s> g(new (std::nothrow) tsmm_graph_s());
    if (e == hipSuccess && g) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch_batched(p->dtype, static_cast<const BatchDesc *>(p->d_desc),
                                       static_cast<const int64_t *>(p->d_inst_start), p->n_work,
                                       p->tile.chunk_rows, static_cast<int32_t *>(p->d_ctr), p->grid, p->block, p->batch_lds, cs);
        e = hipStreamEndCapture(cs, &g->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || !g) {
        if (g && g->graph) (void)hipGraphDestroy(g->graph);
        return g ? hip_fail(e, "graph capture") : fail(TSMM_ERROR_OUT_OF_MEMORY, "host allocation failed");
    }
    g->plan = p;
    ++p->graphs;
    *out = g.release();
    return TSMM_SUCCESS;
}

tsmm_status tsmm_graph_launch(tsmm_graph_t g, void *stream) {
    g_err.clear();
    if (!g || !g->exec) return fail(TSMM_ERROR_INVALID_VALUE, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TSMM_SUCCESS : hip_fail(e, "graph launch");
}

void tsmm_graph_destroy(tsmm_graph_t g) {
    if (!g) return;
    if (g->plan) --g->plan->graphs;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
