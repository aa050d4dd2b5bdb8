// Host side of the C ABI declared in include/lsp.h: spline recognition,
// argument validation, volume storage and kernel dispatch.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lsp.h"
#include "lsp_launch.h"
#include "lsp_backward.h"
#include "lsp_batch.h"
#include "lsp_binned.h"
#include "lsp_plugin.h"
#include "generated/all.h"

namespace {

thread_local std::string g_err;

lsp_status fail(lsp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

lsp_status hip_fail(hipError_t e, const char* what) {
    return fail(LSP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ----------------------------------------------------------- lattices

typedef long long i64;

i64 det3(const i64 m[3][3]) {
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
           m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

// adj(m) with m * adj(m) = det(m) I
void adj3(const i64 m[3][3], i64 a[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            a[i][j] = m[r0][c0] * m[r1][c1] - m[r0][c1] * m[r1][c0];
        }
}

// L Z^3 == R Z^3  iff  |det L| == |det R| and L^{-1} R is an integer matrix.
bool same_lattice(const i64 L[3][3], const i64 R[3][3]) {
    const i64 dl = det3(L), dr = det3(R);
    if (dl == 0 || (dl < 0 ? -dl : dl) != (dr < 0 ? -dr : dr)) return false;
    i64 a[3][3];
    adj3(L, a);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            i64 v = 0;
            for (int k = 0; k < 3; ++k) v += a[i][k] * R[k][j];
            if (v % dl != 0) return false;
        }
    return true;
}

// Launch of the evaluation kernels of a spline compiled into a plugin.
using PluginEval = hipError_t (*)(const lsp::EvalArgs*);

struct SplineDef {
    int kind;
    int lattice;                 // 0 Z^3, 1 BCC, 2 FCC
    std::string name;
    PluginEval plugin_eval;      // null for the built-in splines
    i64 L[3][3];                 // columns are generators
    std::vector<std::vector<int>> dirs;  // canonical directions, with repeats
    int n_cosets;
    int D;
    int shift[4][3];
    int taps, union_taps, n_reference, degree, radius, fma_eval, pad;
    int omin, omax;              // per-axis offset range in global axes (lattice units)
    int continuity;              // phi in C^continuity
};

int rank3(const std::vector<std::vector<int>>& v) {
    // rank of a set of integer 3-vectors: 3 if some triple has a nonzero
    // determinant, else 2 if some pair has a nonzero cross product, ...
    const size_t n = v.size();
    for (size_t a = 0; a < n; ++a)
        for (size_t b = a + 1; b < n; ++b)
            for (size_t c = b + 1; c < n; ++c) {
                const i64 d = (i64)v[a][0] * (v[b][1] * v[c][2] - v[b][2] * v[c][1]) -
                              (i64)v[a][1] * (v[b][0] * v[c][2] - v[b][2] * v[c][0]) +
                              (i64)v[a][2] * (v[b][0] * v[c][1] - v[b][1] * v[c][0]);
                if (d) return 3;
            }
    for (size_t a = 0; a < n; ++a)
        for (size_t b = a + 1; b < n; ++b)
            if (v[a][1] * v[b][2] != v[a][2] * v[b][1] || v[a][0] * v[b][2] != v[a][2] * v[b][0] ||
                v[a][0] * v[b][1] != v[a][1] * v[b][0])
                return 2;
    for (const auto& x : v)
        if (x[0] || x[1] || x[2]) return 1;
    return 0;
}

// A box spline is C^(m-2) where m is the fewest directions whose removal
// leaves a set that does not span the space.
int box_continuity(const std::vector<std::vector<int>>& dirs) {
    const int n = (int)dirs.size();
    int m = n;
    for (unsigned mask = 1; mask < (1u << n); ++mask) {
        const int k = __builtin_popcount(mask);
        if (k >= m) continue;
        std::vector<std::vector<int>> rest;
        for (int j = 0; j < n; ++j)
            if (!(mask >> j & 1)) rest.push_back(dirs[j]);
        if (rank3(rest) < 3) m = k;
    }
    return m - 2;
}

std::vector<int> canon_dir(std::vector<int> d) {
    int sg = 0;
    for (int v : d)
        if (v) { sg = v > 0 ? 1 : -1; break; }
    for (int& v : d) v *= sg;
    return d;
}

// The host description of a spline, from the description of its generated
// tables (lsp_plugin.h): built-in kinds and plugins alike.
SplineDef def_from_desc(const lsp::SplineDesc& d) {
    SplineDef s{};
    s.kind = d.kind;
    s.lattice = d.lattice;
    s.name = std::string(d.name, strnlen(d.name, sizeof(d.name)));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s.L[i][j] = d.L[i][j];
    for (int k = 0; k < d.n_dirs; ++k)
        s.dirs.push_back(canon_dir({d.dirs[k][0], d.dirs[k][1], d.dirs[k][2]}));
    s.n_cosets = d.n_cosets;
    s.D = d.D;
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 3; ++a) s.shift[m][a] = d.shift[m][a];
    s.union_taps = d.union_taps;
    s.taps = d.taps;
    s.n_reference = d.n_reference;
    s.degree = d.degree;
    s.radius = d.radius;
    s.fma_eval = d.fma_eval;
    // per-axis range of stencil offsets in global axes: reflections and
    // permutations make it the symmetric [-radius, radius]
    s.omin = d.symmetry == lsp::kSymNone ? d.off_lo : -s.radius;
    s.omax = d.symmetry == lsp::kSymNone ? d.off_hi : s.radius;
    // an active point's taps reach at most 2 * radius lattice units outside
    // the stored range: ceil(2 radius / D) sites, plus one
    s.pad = (2 * s.radius + s.D - 1) / s.D + 1;
    s.continuity = box_continuity(s.dirs);
    return s;
}

template <int K>
SplineDef make_def() {
    lsp::SplineDesc d;
    lsp::describe<K>(&d);
    return def_from_desc(d);
}

const std::vector<SplineDef>& defs() {
    static const std::vector<SplineDef> v = [] {
        std::vector<SplineDef> out;
#define LSP_DEF(k) out.push_back(make_def<k>());
        LSP_FOR_EACH_KIND(LSP_DEF)
#undef LSP_DEF
        return out;
    }();
    return v;
}

int elem_size(int ctype) { return ctype == lsp::kCF32 ? 4 : 2; }

// Dynamic LDS per evaluation workgroup, read once from LSP_EVAL_LDS (bytes):
// a tuning knob that lowers occupancy (fewer waves share each CU's L1).
// FCC 6-direction: evaluate both reference polynomials and select
// (LSP_FCC_PREDICATED=1) instead of branching on the sub-region.
// Largest point count evaluated with four lanes per point by the separable
// splines (LSP_OPT_SPLIT_MAXN, else LSP_SPLIT_MAXN in the environment; -1
// when neither is set: each spline's measured default).
std::atomic<int> g_opt_split{-2};

int split_maxn() {
    const int o = g_opt_split.load(std::memory_order_relaxed);
    if (o >= -1) return o;
    static const int v = [] {
        const char* env = getenv("LSP_SPLIT_MAXN");
        if (!env) return -1;
        const long x = strtol(env, nullptr, 10);
        return (int)(x < 0 ? 0 : (x > 0x7fffffffL ? 0x7fffffffL : x));
    }();
    return v;
}

// Branch-free evaluation of splines with two reference polynomials
// (LSP_OPT_PREDICATED; -1: not set, the environment's LSP_FCC_PREDICATED).
std::atomic<int> g_opt_pred{-1};

bool fcc_predicated() {
    const int o = g_opt_pred.load(std::memory_order_relaxed);
    if (o >= 0) return o == 1;
    static const bool v = [] {
        const char* env = getenv("LSP_FCC_PREDICATED");
        return env && env[0] == '1';
    }();
    return v;
}

// Matrix-core evaluation for splines that have it: LSP_OPT_MFMA (0 never,
// 1 always, 2 for 16-bit coefficient storage), default from LSP_MFMA, else 0.
std::atomic<int> g_opt_mfma{-1};

bool mfma_for(int ctype) {
    int o = g_opt_mfma.load(std::memory_order_relaxed);
    if (o < 0) {
        static const int v = [] {
            const char* env = getenv("LSP_MFMA");
            const int x = env ? atoi(env) : 0;
            return x < 0 || x > 2 ? 0 : x;
        }();
        o = v;
    }
    return o == 1 || (o == 2 && ctype != lsp::kCF32);
}

unsigned eval_lds_bytes() {
    static const unsigned v = [] {
        const char* env = getenv("LSP_EVAL_LDS");
        long x = env ? strtol(env, nullptr, 10) : 0;
        return (unsigned)(x < 0 ? 0 : (x > 65536 ? 65536 : x));
    }();
    return v;
}

int ctype_of(lsp_dtype storage) {
    switch (storage) {
        case LSP_F32: return lsp::kCF32;
        case LSP_BF16: return lsp::kCBF16;
        case LSP_F16: return lsp::kCF16;
        default: return -1;
    }
}

lsp_status fail(lsp_status st, const char* fmt, ...);

// Brick extent (x, y, z) of the interleaved layout per lattice and element
// size: one brick is one 128-byte line (cosets interleaved), in the shapes
// that minimise the lines a random point's stencil touches.
// LSP_BRICK="bx,by,bz" overrides them.
void brick_dims(int lattice, int es, int b[3]) {
    static const int tab[3][2][3] = {
        {{2, 4, 4}, {4, 4, 4}},   // Z^3 (1 coset per site): 4-byte, 2-byte coefficients
        {{2, 2, 4}, {4, 4, 2}},   // BCC (2 cosets per site)
        {{2, 2, 2}, {2, 4, 2}},   // FCC (4 cosets per site)
    };
    const int l = (lattice < 0 || lattice > 2) ? 0 : lattice;
    for (int a = 0; a < 3; ++a) b[a] = tab[l][es == 4 ? 0 : 1][a];
    const char* env = getenv("LSP_BRICK");
    int v[3];
    if (env && sscanf(env, "%d,%d,%d", &v[0], &v[1], &v[2]) == 3) {
        bool ok = true;
        for (int a = 0; a < 3; ++a) ok = ok && v[a] >= 1 && v[a] <= 64 && (v[a] & (v[a] - 1)) == 0;
        if (ok)
            for (int a = 0; a < 3; ++a) b[a] = v[a];
    }
}

// Internal layout of a volume (interleaved cosets, bricks, zero halo) and the
// range of ROE lattice points whose stencil reaches a stored site.
lsp_status make_geom(const SplineDef& d, const int64_t dims[3], int ctype, lsp::VolGeom* out,
                     size_t* nbytes) {
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > (1 << 20))
            return fail(LSP_E_SHAPE, "dims[%d] = %lld out of [1, 2^20]", a, (long long)dims[a]);
    const int es = elem_size(ctype);
    int br[3];
    brick_dims(d.lattice, es, br);
    const i64 site = (i64)d.n_cosets * es;
    i64 nb[3];
    for (int a = 0; a < 3; ++a) nb[a] = (dims[a] + 2 * d.pad + br[a] - 1) / br[a];
    const i64 brick = (i64)br[0] * br[1] * br[2] * site;
    const i64 total = nb[0] * nb[1] * nb[2] * brick;
    if (total >= ((i64)1 << 31))
        return fail(LSP_E_SHAPE, "padded coefficient buffer of %lld bytes exceeds 2^31", (long long)total);
    lsp::VolGeom g{};
    g.es = es;
    g.pad = d.pad;
    for (int a = 0; a < 3; ++a) {
        int l = 0;
        while ((1 << l) < br[a]) ++l;
        g.lb[a] = l;
    }
    if (nb[0] * nb[1] >= ((i64)1 << 24))
        return fail(LSP_E_SHAPE, "%lld x %lld bricks per slab exceed 2^24", (long long)nb[0],
                    (long long)nb[1]);
    auto log2i = [](i64 v) { int l = 0; while (((i64)1 << l) < v) ++l; return l; };
    g.lis[0] = log2i(site);
    g.lis[1] = log2i(br[0] * site);
    g.lis[2] = log2i(br[0] * br[1] * site);
    g.nbs[0] = 1;
    g.nbs[1] = (int)nb[0];
    g.nbs[2] = (int)(nb[0] * nb[1]);
    g.lbb = log2i(brick);
    for (int a = 0; a < 3; ++a) {
        int shmax = 0;
        for (int m = 0; m < d.n_cosets; ++m) shmax = std::max(shmax, d.shift[m][a]);
        const i64 maxsite = (i64)d.D * (dims[a] - 1) + shmax;
        // some tap k + o (o in [omin, omax]) lies in [0, maxsite]
        g.kmin[a] = -d.omax;
        g.kmax[a] = (int)(maxsite - d.omin);
    }
    *out = g;
    *nbytes = (size_t)total;
    return LSP_OK;
}
}  // namespace

struct lsp_spline {
    SplineDef def;
};

struct lsp_volume {
    SplineDef def;
    int64_t dims[3];
    lsp_dtype storage;
    int ctype;
    void* buf;
    size_t nbytes;
    int device;
    lsp::VolGeom geom;
};

extern "C" {

const char* lsp_status_string(lsp_status st) {
    switch (st) {
        case LSP_OK: return "ok";
        case LSP_E_INVALID_ARG: return "invalid argument";
        case LSP_E_UNSUPPORTED: return "unsupported spline";
        case LSP_E_DTYPE: return "unsupported dtype";
        case LSP_E_SHAPE: return "size out of range";
        case LSP_E_WORKSPACE: return "workspace too small";
        case LSP_E_HIP: return "HIP error";
        case LSP_E_OOM: return "out of device memory";
    }
    return "unknown status";
}

const char* lsp_last_error(void) { return g_err.c_str(); }

lsp_status lsp_set_option(int option, int value) {
    if (option == LSP_OPT_MFMA) {
        if (value < 0 || value > 2) return fail(LSP_E_INVALID_ARG, "LSP_OPT_MFMA takes 0, 1 or 2");
        g_opt_mfma.store(value, std::memory_order_relaxed);
        return LSP_OK;
    }
    if (option == LSP_OPT_SPLIT_MAXN) {
        if (value < -1) return fail(LSP_E_INVALID_ARG, "LSP_OPT_SPLIT_MAXN takes a count >= 0, or -1");
        g_opt_split.store(value, std::memory_order_relaxed);
        return LSP_OK;
    }
    if (option == LSP_OPT_PREDICATED) {
        if (value < 0 || value > 1) return fail(LSP_E_INVALID_ARG, "LSP_OPT_PREDICATED takes 0 or 1");
        g_opt_pred.store(value, std::memory_order_relaxed);
        return LSP_OK;
    }
    return fail(LSP_E_INVALID_ARG, "unknown option %d", option);
}

const char* lsp_version(void) { return "lsp 0.1 (gfx950)"; }

lsp_status lsp_spline_create(int s, const int32_t* L, const int32_t* Xi, int n_dirs,
                             lsp_spline** out) {
    if (!out) return fail(LSP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!L || !Xi) return fail(LSP_E_INVALID_ARG, "L or Xi is NULL");
    if (s != 3) return fail(LSP_E_UNSUPPORTED, "only s = 3 is supported (got %d)", s);
    if (n_dirs < 3 || n_dirs > 64) return fail(LSP_E_INVALID_ARG, "n_dirs %d out of [3, 64]", n_dirs);
    i64 Lm[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Lm[i][j] = L[i * 3 + j];
    if (det3(Lm) == 0) return fail(LSP_E_INVALID_ARG, "L is singular");
    std::vector<std::vector<int>> dirs;
    for (int j = 0; j < n_dirs; ++j) {
        std::vector<int> d = {Xi[0 * n_dirs + j], Xi[1 * n_dirs + j], Xi[2 * n_dirs + j]};
        if (d[0] == 0 && d[1] == 0 && d[2] == 0)
            return fail(LSP_E_INVALID_ARG, "direction %d is zero", j);
        dirs.push_back(canon_dir(d));
    }
    std::sort(dirs.begin(), dirs.end());
    for (const SplineDef& d : defs()) {
        std::vector<std::vector<int>> want = d.dirs;
        std::sort(want.begin(), want.end());
        if (want == dirs && same_lattice(Lm, d.L)) {
            lsp_spline* sp = new (std::nothrow) lsp_spline;
            if (!sp) return fail(LSP_E_OOM, "host allocation failed");
            sp->def = d;
            *out = sp;
            return LSP_OK;
        }
    }
    return fail(LSP_E_UNSUPPORTED,
                "no generated code for this (L, Xi): supported are the trilinear, triquadratic, "
                "tricubic, 6-direction and 7-direction box splines on Z^3, the BCC 4-, 7- and "
                "8-direction and the FCC 6-direction box splines");
}

lsp_status lsp_spline_load_plugin(const char* path, lsp_spline** out) {
    if (!out) return fail(LSP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!path) return fail(LSP_E_INVALID_ARG, "path is NULL");
    // kept loaded until the process ends: its kernels back every volume of the spline
    void* h = dlopen(path, RTLD_NOW | RTLD_LOCAL);
    if (!h) return fail(LSP_E_UNSUPPORTED, "cannot load %s: %s", path, dlerror());
    using Describe = int (*)(lsp::SplineDesc*);
    auto describe = reinterpret_cast<Describe>(dlsym(h, "lsp_plugin_describe"));
    auto eval = reinterpret_cast<PluginEval>(dlsym(h, "lsp_plugin_eval"));
    if (!describe || !eval) return fail(LSP_E_UNSUPPORTED, "%s exports no spline plugin entry points", path);
    lsp::SplineDesc d{};
    if (describe(&d) != 0 || d.abi != lsp::kPluginAbi)
        return fail(LSP_E_UNSUPPORTED, "%s was built for another library version (ABI %x, expected %x)", path,
                    (unsigned)d.abi, (unsigned)lsp::kPluginAbi);
    if (d.n_dirs < 3 || d.n_dirs > lsp::kDescMaxDirs || d.n_cosets < 1 || d.n_cosets > 4 ||
        d.lattice < 0 || d.lattice > 2)
        return fail(LSP_E_UNSUPPORTED, "%s describes an unsupported spline", path);
    lsp_spline* sp = new (std::nothrow) lsp_spline;
    if (!sp) return fail(LSP_E_OOM, "host allocation failed");
    sp->def = def_from_desc(d);
    sp->def.plugin_eval = eval;
    *out = sp;
    return LSP_OK;
}

void lsp_spline_destroy(lsp_spline* sp) { delete sp; }

static void fill_info(const SplineDef& d, lsp_spline_info* o) {
    memset(o, 0, sizeof(*o));
    o->s = 3;
    o->kind = d.kind;
    o->n_cosets = d.n_cosets;
    for (int a = 0; a < 3; ++a) o->D[a] = d.D;
    memcpy(o->shift, d.shift, sizeof(o->shift));
    o->taps = d.taps;
    o->union_taps = d.union_taps;
    o->n_reference = d.n_reference;
    o->degree = d.degree;
    o->radius = d.radius;
    o->fma_eval = d.fma_eval;
    o->pad = d.pad;
    o->continuity = d.continuity;
}

lsp_status lsp_spline_get_info(const lsp_spline* sp, lsp_spline_info* out) {
    if (!sp || !out) return fail(LSP_E_INVALID_ARG, "NULL argument");
    fill_info(sp->def, out);
    return LSP_OK;
}

lsp_status lsp_volume_create(const lsp_spline* sp, const int64_t dims[3], lsp_dtype storage,
                             lsp_volume** out) {
    if (!out) return fail(LSP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!sp || !dims) return fail(LSP_E_INVALID_ARG, "NULL argument");
    const int ctype = ctype_of(storage);
    if (ctype < 0) return fail(LSP_E_DTYPE, "storage dtype must be F32, BF16 or F16");
    const SplineDef& d = sp->def;
    lsp::VolGeom g{};
    size_t total = 0;
    lsp_status st = make_geom(d, dims, ctype, &g, &total);
    if (st) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void* buf = nullptr;
    e = hipMalloc(&buf, (size_t)total);
    if (e != hipSuccess) return fail(LSP_E_OOM, "hipMalloc(%lld): %s", (long long)total, hipGetErrorString(e));
    e = hipMemset(buf, 0, (size_t)total);
    if (e != hipSuccess) {
        (void)hipFree(buf);
        return hip_fail(e, "hipMemset");
    }
    lsp_volume* v = new (std::nothrow) lsp_volume;
    if (!v) {
        (void)hipFree(buf);
        return fail(LSP_E_OOM, "host allocation failed");
    }
    v->def = d;
    memcpy(v->dims, dims, sizeof(v->dims));
    v->storage = storage;
    v->ctype = ctype;
    v->buf = buf;
    v->nbytes = (size_t)total;
    v->device = dev;
    v->geom = g;
    *out = v;
    return LSP_OK;
}

void lsp_volume_destroy(lsp_volume* vol) {
    if (!vol) return;
    if (vol->buf) (void)hipFree(vol->buf);
    delete vol;
}

lsp_status lsp_volume_info(const lsp_volume* vol, lsp_spline_info* spline, int64_t dims[3],
                           lsp_dtype* storage) {
    if (!vol) return fail(LSP_E_INVALID_ARG, "vol is NULL");
    if (spline) fill_info(vol->def, spline);
    if (dims) memcpy(dims, vol->dims, sizeof(vol->dims));
    if (storage) *storage = vol->storage;
    return LSP_OK;
}

lsp_status lsp_volume_set_coeffs(lsp_volume* vol, const void* const* coset_ptrs, lsp_dtype src,
                                 hipStream_t stream) {
    if (!vol || !coset_ptrs) return fail(LSP_E_INVALID_ARG, "NULL argument");
    if (src != LSP_F32 && src != LSP_F64 && src != LSP_BF16 && src != LSP_F16)
        return fail(LSP_E_DTYPE, "source dtype %d not supported", (int)src);
    for (int m = 0; m < vol->def.n_cosets; ++m)
        if (!coset_ptrs[m]) return fail(LSP_E_INVALID_ARG, "coset_ptrs[%d] is NULL", m);
    for (int m = 0; m < vol->def.n_cosets; ++m) {
        hipError_t e = lsp::launch_pack(coset_ptrs[m], (int)src, vol->ctype, vol->buf, vol->dims,
                                        vol->geom, m, stream);
        if (e != hipSuccess) return hip_fail(e, "pack kernel launch");
    }
    return LSP_OK;
}

static lsp_status check_eval_args(const lsp_volume* vol, const void* pts, lsp_dtype pd, int64_t N) {
    if (!vol) return fail(LSP_E_INVALID_ARG, "vol is NULL");
    if (N < 0 || N >= ((int64_t)1 << 31)) return fail(LSP_E_SHAPE, "N = %lld out of [0, 2^31)", (long long)N);
    if (pd != LSP_F32 && pd != LSP_F64) return fail(LSP_E_DTYPE, "points must be F32 or F64");
    if (N > 0 && !pts) return fail(LSP_E_INVALID_ARG, "pts is NULL");
    return LSP_OK;
}

static lsp_status run_eval(const lsp_volume* vol, const void* pts, lsp_dtype pd, int64_t N,
                           int mode, float* out, float* grad, const float* gin, hipStream_t stream,
                           float* hess = nullptr) {
    lsp::EvalArgs a{};
    a.kind = vol->def.kind;
    a.ctype = vol->ctype;
    a.pts_f64 = pd == LSP_F64;
    a.mode = mode;
    a.predicated = fcc_predicated();
    a.pts = pts;
    a.N = (int)N;
    a.coef = vol->buf;
    a.nbytes = (unsigned)vol->nbytes;
    a.g = vol->geom;
    a.out = out;
    a.grad = grad;
    a.gin = gin;
    a.hess = hess;
    a.stream = stream;
    a.lds_bytes = eval_lds_bytes();
    a.mfma = mfma_for(vol->ctype);
    a.split_maxn = split_maxn();
    hipError_t e = hipSuccess;
    bool found = false;
    if (vol->def.plugin_eval) {
        e = a.N > 0 ? vol->def.plugin_eval(&a) : hipSuccess;
        found = true;
    }
#define LSP_RUN(k) \
    if (!found && a.kind == k) { e = lsp::launch_eval<k>(a); found = true; }
    LSP_FOR_EACH_KIND(LSP_RUN)
#undef LSP_RUN
    if (!found) return fail(LSP_E_UNSUPPORTED, "kind %d", a.kind);
    if (e != hipSuccess) return hip_fail(e, "evaluation kernel launch");
    return LSP_OK;
}

lsp_status lsp_eval(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                    float* out, hipStream_t stream) {
    lsp_status st = check_eval_args(vol, pts, pts_dtype, N);
    if (st) return st;
    if (N > 0 && !out) return fail(LSP_E_INVALID_ARG, "out is NULL");
    return run_eval(vol, pts, pts_dtype, N, lsp::kValue, out, nullptr, nullptr, stream);
}

lsp_status lsp_eval_grad(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                         float* val, float* grad, hipStream_t stream) {
    lsp_status st = check_eval_args(vol, pts, pts_dtype, N);
    if (st) return st;
    if (N > 0 && !grad) return fail(LSP_E_INVALID_ARG, "grad is NULL");
    return run_eval(vol, pts, pts_dtype, N, lsp::kValueGrad, val, grad, nullptr, stream);
}

lsp_status lsp_eval_hessian(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype,
                            int64_t N, float* val, float* grad, float* hess, hipStream_t stream) {
    lsp_status st = check_eval_args(vol, pts, pts_dtype, N);
    if (st) return st;
    if (vol->def.continuity < 1)
        return fail(LSP_E_UNSUPPORTED, "%s is only C^%d: no second derivatives", vol->def.name.c_str(),
                    vol->def.continuity);
    if (N > 0 && !hess) return fail(LSP_E_INVALID_ARG, "hess is NULL");
    return run_eval(vol, pts, pts_dtype, N, lsp::kValueGradHess, val, grad, nullptr, stream, hess);
}

// Bin extent 2^lb coset units: the smallest lb >= LSP_BIN_LB (default 3)
// with at most kMaxBins bins.
static lsp::BinGeom bin_geom(const lsp_volume* vol) {
    static const int lb0 = [] {
        const char* env = getenv("LSP_BIN_LB");
        const int v = env ? atoi(env) : 3;
        return v < 1 ? 1 : (v > 8 ? 8 : v);
    }();
    lsp::BinGeom bg{};
    int64_t P[3];
    for (int a = 0; a < 3; ++a) P[a] = vol->dims[a] + 2 * vol->def.pad;
    for (bg.lb = lb0;; ++bg.lb) {
        int64_t n = 1;
        for (int a = 0; a < 3; ++a) {
            bg.nb[a] = (int)((P[a] + (1 << bg.lb) - 1) >> bg.lb);
            n *= bg.nb[a];
        }
        if (n <= lsp::kMaxBins) {
            bg.nbins = (int)n;
            break;
        }
    }
    return bg;
}

lsp_status lsp_eval_binned_workspace_size(const lsp_volume* vol, lsp_dtype pts_dtype, int64_t N,
                                          size_t* bytes) {
    lsp_status st = check_eval_args(vol, (const void*)1, pts_dtype, N);
    if (st) return st;
    if (vol->def.plugin_eval) return fail(LSP_E_UNSUPPORTED, "binned order: built-in splines only");
    if (!bytes) return fail(LSP_E_INVALID_ARG, "bytes is NULL");
    *bytes = lsp::binned_workspace_bytes(bin_geom(vol), (int)N, pts_dtype == LSP_F64);
    return LSP_OK;
}

lsp_status lsp_eval_binned(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                           float* val, float* grad, void* workspace, size_t ws_bytes,
                           hipStream_t stream) {
    lsp_status st = check_eval_args(vol, pts, pts_dtype, N);
    if (st) return st;
    if (vol->def.plugin_eval) return fail(LSP_E_UNSUPPORTED, "binned order: built-in splines only");
    if (N > 0 && !val) return fail(LSP_E_INVALID_ARG, "val is NULL");
    if (N == 0) return LSP_OK;
    lsp::BinnedArgs a{};
    a.bg = bin_geom(vol);
    const size_t need = lsp::binned_workspace_bytes(a.bg, (int)N, pts_dtype == LSP_F64);
    if (!workspace || ws_bytes < need)
        return fail(LSP_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (((uintptr_t)workspace & 255) != 0) return fail(LSP_E_WORKSPACE, "workspace must be 256-byte aligned");
    a.kind = vol->def.kind;
    a.ctype = vol->ctype;
    a.pts_f64 = pts_dtype == LSP_F64;
    a.pts = pts;
    a.N = (int)N;
    a.coef = vol->buf;
    a.nbytes = (unsigned)vol->nbytes;
    a.g = vol->geom;
    a.out = val;
    a.grad = grad;
    a.ws = workspace;
    a.ws_bytes = ws_bytes;
    a.stream = stream;
    a.mfma = mfma_for(vol->ctype);
    a.split_maxn = split_maxn();
    hipError_t e = lsp::launch_binned(a);
    if (e != hipSuccess) return hip_fail(e, "binned evaluation launch");
    return LSP_OK;
}

lsp_status lsp_backward_workspace_size(const lsp_volume* vol, int64_t N, size_t* bytes) {
    if (!vol || !bytes) return fail(LSP_E_INVALID_ARG, "NULL argument");
    if (N < 0 || N >= ((int64_t)1 << 31)) return fail(LSP_E_SHAPE, "N = %lld out of [0, 2^31)", (long long)N);
    if (vol->def.plugin_eval) return fail(LSP_E_UNSUPPORTED, "dL/dc: built-in splines only");
    const size_t b = lsp::backward_workspace_bytes(vol->def.kind, vol->def.n_cosets, vol->dims,
                                                   vol->def.pad, N);
    if (b == (size_t)-1) return fail(LSP_E_HIP, "sort workspace query failed");
    *bytes = b;
    return LSP_OK;
}

lsp_status lsp_backward(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                        const float* dL_df, float* dL_dc, float* dL_dx, void* workspace,
                        size_t ws_bytes, hipStream_t stream) {
    lsp_status st = check_eval_args(vol, pts, pts_dtype, N);
    if (st) return st;
    if (N > 0 && !dL_df && (dL_dc || dL_dx)) return fail(LSP_E_INVALID_ARG, "dL_df is NULL");
    if (dL_dc && vol->def.plugin_eval) return fail(LSP_E_UNSUPPORTED, "dL/dc: built-in splines only");
    if (dL_dx && N > 0) {
        st = run_eval(vol, pts, pts_dtype, N, lsp::kGradX, nullptr, dL_dx, dL_df, stream);
        if (st) return st;
    }
    if (dL_dc) {
        const size_t need = lsp::backward_workspace_bytes(vol->def.kind, vol->def.n_cosets, vol->dims,
                                                          vol->def.pad, N);
        if (need == (size_t)-1) return fail(LSP_E_HIP, "sort workspace query failed");
        if (need > 0 && (!workspace || ws_bytes < need))
            return fail(LSP_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
        if (((uintptr_t)workspace & 255) != 0)
            return fail(LSP_E_WORKSPACE, "workspace must be 256-byte aligned");
        lsp::BackwardArgs b{};
        b.kind = vol->def.kind;
        b.ctype = vol->ctype;
        b.pts_f64 = pts_dtype == LSP_F64;
        b.pts = pts;
        b.N = (int)N;
        b.g = vol->geom;
        b.n_cosets = vol->def.n_cosets;
        for (int a = 0; a < 3; ++a) b.dims[a] = (int)vol->dims[a];
        b.dL_df = dL_df;
        b.dL_dc = dL_dc;
        b.ws = workspace;
        b.ws_bytes = ws_bytes;
        b.stream = stream;
        hipError_t e = lsp::launch_backward_coef(b);
        if (e != hipSuccess) return hip_fail(e, "backward kernel launch");
    }
    return LSP_OK;
}

lsp_status lsp_backward_dx_from_grad(int64_t N, const float* dL_df, const float* grad_f,
                                     float* dL_dx, hipStream_t stream) {
    if (N < 0) return fail(LSP_E_SHAPE, "N < 0");
    if (N > 0 && (!dL_df || !grad_f || !dL_dx)) return fail(LSP_E_INVALID_ARG, "NULL array");
    hipError_t e = lsp::launch_dx_from_grad(N, dL_df, grad_f, dL_dx, stream);
    if (e != hipSuccess) return hip_fail(e, "dL/dx launch");
    return LSP_OK;
}

// ------------------------------------------------------------ batched plans

}  // extern "C"

struct lsp_batch_plan {
    int n_vol = 0;
    int n_items = 0;
    int tile = 0;
    int blocks = 0;
    int device = 0;
    lsp::BatchVol* d_vols = nullptr;
    lsp::BatchItem* d_items = nullptr;
    std::vector<lsp::BatchGroup> groups;   // host copy, launch order
    int* d_counter = nullptr;              // one per group
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune_cache;  // signature -> (tile, blocks/CU)

// Items grouped by kernel variant (kind, storage, value / value+gradient),
// groups with the most points first; inside a group the largest volumes
// first, so their many tiles are handed out before the tail.
std::vector<lsp::BatchItem> make_items(const std::vector<lsp::BatchVol>& hv, int tile,
                                       std::vector<lsp::BatchGroup>* groups) {
    auto key = [&](int v) { return (hv[v].kind * 3 + hv[v].ctype) * 2 + (hv[v].grad ? 1 : 0); };
    std::map<int, long long> work;
    for (size_t v = 0; v < hv.size(); ++v) work[key((int)v)] += hv[v].N;
    std::vector<int> order(hv.size());
    for (size_t v = 0; v < hv.size(); ++v) order[v] = (int)v;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ka = key(a), kb = key(b);
        if (ka != kb) return work[ka] != work[kb] ? work[ka] > work[kb] : ka < kb;
        return hv[a].N > hv[b].N;
    });
    std::vector<lsp::BatchItem> items;
    groups->clear();
    int cur = -1;
    for (int v : order) {
        if (hv[v].N == 0) continue;
        if (key(v) != cur) {
            cur = key(v);
            groups->push_back({hv[v].kind, hv[v].ctype, hv[v].grad ? 1 : 0, (int)items.size(), 0});
        }
        for (long long s = 0; s < hv[v].N; s += tile)
            items.push_back({v, (int)s, (int)std::min<long long>(tile, hv[v].N - s)});
        groups->back().count = (int)items.size() - groups->back().first;
    }
    return items;
}

void destroy_plan(lsp_batch_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->d_vols) (void)hipFree(p->d_vols);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_counter) (void)hipFree(p->d_counter);
    delete p;
}

lsp_status upload_items(lsp_batch_plan* p, const std::vector<lsp::BatchItem>& items) {
    if (p->d_items) (void)hipFree(p->d_items);
    p->d_items = nullptr;
    p->n_items = (int)items.size();
    if (items.empty()) return LSP_OK;
    hipError_t e = hipMalloc(&p->d_items, sizeof(lsp::BatchItem) * items.size());
    if (e != hipSuccess) return fail(LSP_E_OOM, "hipMalloc(items): %s", hipGetErrorString(e));
    e = hipMemcpy(p->d_items, items.data(), sizeof(lsp::BatchItem) * items.size(),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(items)");
    return LSP_OK;
}

}  // namespace

extern "C" {

lsp_status lsp_batch_plan_create(int n_vol, const lsp_volume* const* vols, const float* const* pts,
                                 const int64_t* N, float* const* val, float* const* grad, int flags,
                                 hipStream_t stream, lsp_batch_plan** out) {
    if (!out) return fail(LSP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_vol < 1 || n_vol > (1 << 16)) return fail(LSP_E_SHAPE, "n_vol %d out of [1, 65536]", n_vol);
    if (!vols || !pts || !N || !val) return fail(LSP_E_INVALID_ARG, "NULL array argument");
    std::vector<lsp::BatchVol> hv(n_vol);
    long long total = 0;
    for (int v = 0; v < n_vol; ++v) {
        const lsp_volume* vol = vols[v];
        if (!vol) return fail(LSP_E_INVALID_ARG, "vols[%d] is NULL", v);
        if (vol->def.plugin_eval) return fail(LSP_E_UNSUPPORTED, "vols[%d]: batch plans take built-in splines only", v);
        if (N[v] < 0 || N[v] >= ((int64_t)1 << 31)) return fail(LSP_E_SHAPE, "N[%d] out of range", v);
        const bool want_grad = grad && grad[v];
        if (N[v] > 0 && (!pts[v] || (!val[v] && !want_grad)))
            return fail(LSP_E_INVALID_ARG, "volume %d: pts or outputs are NULL", v);
        lsp::BatchVol& b = hv[v];
        b.coef = vol->buf;
        b.nbytes = (unsigned)vol->nbytes;
        b.kind = vol->def.kind;
        b.ctype = vol->ctype;
        b.N = (int)N[v];
        b.g = vol->geom;
        b.pts = pts[v];
        b.val = val[v];
        b.grad = want_grad ? grad[v] : nullptr;
        total += N[v];
    }
    lsp_batch_plan* p = new (std::nothrow) lsp_batch_plan;
    if (!p) return fail(LSP_E_OOM, "host allocation failed");
    p->n_vol = n_vol;
    hipError_t e = hipGetDevice(&p->device);
    int ncu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "device query"); }
    e = hipMalloc(&p->d_vols, sizeof(lsp::BatchVol) * n_vol);
    // one counter per possible variant (kinds x storages x modes)
    if (e == hipSuccess) e = hipMalloc(&p->d_counter, sizeof(int) * lsp::gen::kNumKinds * 3 * 2);
    if (e != hipSuccess) { destroy_plan(p); return fail(LSP_E_OOM, "hipMalloc: %s", hipGetErrorString(e)); }
    // every launch leaves its counters at zero again, so they are set once
    e = lsp::reset_batch_counters(p->d_counter, lsp::gen::kNumKinds * 3 * 2, stream);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "counter reset"); }
    e = hipMemcpy(p->d_vols, hv.data(), sizeof(lsp::BatchVol) * n_vol, hipMemcpyHostToDevice);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "hipMemcpy(vols)"); }

    // signature of the batch for the tuning cache: kinds, storage, modes, sizes
    const int smax = split_maxn();
    std::string sig = std::to_string(ncu) + ":" + std::to_string(smax) + ":";
    for (const lsp::BatchVol& b : hv)
        sig += std::to_string(b.kind) + "/" + std::to_string(b.ctype) + "/" + (b.grad ? "g" : "v") +
               "/" + std::to_string(b.N) + "/" + std::to_string(b.nbytes) + ";";
    int tile = 4096, bpc = 8;
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(sig);
        if (it != g_tune_cache.end()) { tile = it->second.first; bpc = it->second.second; cached = true; }
    }
    if ((flags & LSP_BATCH_AUTOTUNE) && !cached && total > 0) {
        // time every candidate launch shape on the caller's stream
        // (256-point tiles let a small batch spread over every CU)
        const int tiles[4] = {256, 1024, 4096, 16384};
        const int bpcs[3] = {2, 4, 8};
        hipEvent_t t0, t1;
        (void)hipEventCreate(&t0);
        (void)hipEventCreate(&t1);
        float best = 1e30f;
        for (int ti = 0; ti < 4; ++ti) {
            std::vector<lsp::BatchItem> items = make_items(hv, tiles[ti], &p->groups);
            lsp_status st = upload_items(p, items);
            if (st) { (void)hipEventDestroy(t0); (void)hipEventDestroy(t1); destroy_plan(p); return st; }
            for (int bi = 0; bi < 3; ++bi) {
                const int blocks = std::max(1, std::min(ncu * bpcs[bi], p->n_items));
                e = lsp::launch_batch(p->d_vols, p->d_items, p->groups.data(), (int)p->groups.size(),
                                      p->d_counter, blocks, smax, stream);
                if (e == hipSuccess) e = hipEventRecord(t0, stream);
                for (int r = 0; r < 3 && e == hipSuccess; ++r)
                    e = lsp::launch_batch(p->d_vols, p->d_items, p->groups.data(),
                                          (int)p->groups.size(), p->d_counter, blocks, smax, stream);
                if (e == hipSuccess) e = hipEventRecord(t1, stream);
                if (e == hipSuccess) e = hipEventSynchronize(t1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                if (e != hipSuccess) {
                    (void)hipEventDestroy(t0);
                    (void)hipEventDestroy(t1);
                    destroy_plan(p);
                    return hip_fail(e, "autotune launch");
                }
                if (ms < best) { best = ms; tile = tiles[ti]; bpc = bpcs[bi]; }
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[sig] = {tile, bpc};
    }
    std::vector<lsp::BatchItem> items = make_items(hv, tile, &p->groups);
    lsp_status st = upload_items(p, items);
    if (st) { destroy_plan(p); return st; }
    p->tile = tile;
    p->blocks = std::max(1, std::min(ncu * bpc, std::max(p->n_items, 1)));
    // capture the persistent kernels into a graph on a private stream
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t el = lsp::launch_batch(p->d_vols, p->d_items, p->groups.data(),
                                          (int)p->groups.size(), p->d_counter, p->blocks, smax, p->cap);
        e = hipStreamEndCapture(p->cap, &p->graph);
        if (e == hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "graph capture"); }
    *out = p;
    return LSP_OK;
}

lsp_status lsp_batch_plan_info(const lsp_batch_plan* p, int* tile, int* blocks, int* n_items) {
    if (!p) return fail(LSP_E_INVALID_ARG, "plan is NULL");
    if (tile) *tile = p->tile;
    if (blocks) *blocks = p->blocks;
    if (n_items) *n_items = p->n_items;
    return LSP_OK;
}

lsp_status lsp_batch_run(lsp_batch_plan* p, hipStream_t stream) {
    if (!p || !p->exec) return fail(LSP_E_INVALID_ARG, "plan is NULL");
    hipError_t e = hipGraphLaunch(p->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return LSP_OK;
}

void lsp_batch_plan_destroy(lsp_batch_plan* p) { destroy_plan(p); }

// ------------------------------------------------------------ diagnostics

}  // extern "C"

template <int K>
static void debug_offsets(const lsp::VolGeom& geom, const double* pts, int64_t N, int32_t* offs,
                          int32_t* flags) {
    using T = lsp::TablesOf<K>;
    for (int64_t i = 0; i < N; ++i) {
        float xf[3] = {(float)pts[3 * i], (float)pts[3 * i + 1], (float)pts[3 * i + 2]};
        lsp::Loc L;
        lsp::locate<K>(xf, geom, L);
        flags[i] = (L.active ? 1 : 0) | (L.nan ? 2 : 0) | (L.region << 2);
        for (int j = 0; j < T::kTaps; ++j)
            offs[i * T::kTaps + j] =
                lsp::tap_offset<K>(L, T::kOff[j][0], T::kOff[j][1], T::kOff[j][2], T::kParity[j]);
    }
}

extern "C" {

lsp_status lsp_debug_tap_offsets(const lsp_spline* sp, const int64_t dims[3], lsp_dtype storage,
                                 const double* pts, int64_t N, int32_t* offs, int32_t* flags) {
    if (!sp || !dims || (N > 0 && (!pts || !offs || !flags)))
        return fail(LSP_E_INVALID_ARG, "NULL argument");
    const int ctype = ctype_of(storage);
    if (ctype < 0) return fail(LSP_E_DTYPE, "storage dtype must be F32, BF16 or F16");
    lsp::VolGeom geom{};
    size_t nbytes = 0;
    lsp_status st = make_geom(sp->def, dims, ctype, &geom, &nbytes);
    if (st) return st;
    if (sp->def.plugin_eval) return fail(LSP_E_UNSUPPORTED, "built-in splines only");
#define LSP_OFFS(k) \
    if (sp->def.kind == k) debug_offsets<k>(geom, pts, N, offs, flags);
    LSP_FOR_EACH_KIND(LSP_OFFS)
#undef LSP_OFFS
    return LSP_OK;
}

lsp_status lsp_debug_geometry(const lsp_spline* sp, const int64_t dims[3], lsp_dtype storage,
                              int32_t* out, size_t* nbytes) {
    if (!sp || !dims || !out || !nbytes) return fail(LSP_E_INVALID_ARG, "NULL argument");
    const int ctype = ctype_of(storage);
    if (ctype < 0) return fail(LSP_E_DTYPE, "storage dtype must be F32, BF16 or F16");
    lsp::VolGeom g{};
    lsp_status st = make_geom(sp->def, dims, ctype, &g, nbytes);
    if (st) return st;
    int v[20] = {g.es, g.pad, g.kmin[0], g.kmin[1], g.kmin[2], g.kmax[0], g.kmax[1], g.kmax[2],
                 g.lb[0], g.lb[1], g.lb[2], g.nbs[0] << g.lbb, g.nbs[1] << g.lbb, g.nbs[2] << g.lbb,
                 1 << g.lis[0], 1 << g.lis[1], 1 << g.lis[2], ctype, sp->def.n_cosets, 0};
    memcpy(out, v, sizeof(v));
    return LSP_OK;
}

}  // extern "C"
