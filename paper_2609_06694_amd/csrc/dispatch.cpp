// Dispatch map: case key -> kernel family and launch parameters.
//
// The map plays the role of the paper's operator map (Section 4.2): one cell
// per (dimension, stencil shape, radius, precision, boundary, update, grid
// class), each naming the structure that serves the case.  Compiled-in
// defaults cover every legal case; the autotuner overwrites cells in process
// and, when STENCIL_TUNE_CACHE names a file, appends them there so later
// processes start from the tuned entries.
#include <dlfcn.h>

#include <mutex>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>

#include "plan.h"

namespace stk {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

const char* last_error() { return g_err; }

Geom geom_of(const st_problem& p) {
    Geom g;
    g.ndim = p.ndim;
    g.nx = (int)p.n[0];
    g.ny = (int)p.n[1];
    g.nz = (int)p.n[2];
    g.shape = p.shape;
    g.r = p.radius;
    g.dtype = p.dtype;
    g.boundary = p.boundary;
    g.iso = false;
    return g;
}

Geom plan_geom(const st_plan* pl) {
    Geom g = geom_of(pl->prob);
    g.iso = pl->iso;
    return g;
}

CaseKey classify(const st_problem& p) {
    CaseKey k;
    k.ndim = p.ndim;
    k.shape = p.shape;
    k.r = p.radius;
    k.dtype = p.dtype;
    k.boundary = p.boundary;
    k.update = p.update;
    const double cells = (double)p.n[0] * (double)p.n[1] * (double)p.n[2];
    k.size_class = cells <= (double)(1 << 18)   ? 0
                   : cells <= (double)(1 << 20) ? 1
                   : cells <= (double)(1 << 22) ? 2
                   : cells <= (double)(1 << 25) ? 3
                                                : 4;
    int64_t lo = p.n[0], hi = p.n[0];
    for (int a = 1; a < p.ndim; ++a) {
        lo = p.n[a] < lo ? p.n[a] : lo;
        hi = p.n[a] > hi ? p.n[a] : hi;
    }
    // Slabs (longest side >= 4x the shortest) by orientation to the march
    // (the slowest axis: z in 3D, y in 2D): 1 = the march axis is the
    // shortest (few planes or rows), 2 = it is the longest (a long column),
    // 3 = both the thin and the long side lie across it.
    const int64_t nm = p.n[p.ndim - 1];
    k.slab = hi < 4 * lo ? 0 : (nm == lo ? 1 : (nm == hi ? 2 : 3));
    return k;
}

CaseKey reverse_key(const st_problem& p) {
    CaseKey k = classify(p);
    k.update = kKeyWaveReverse;
    return k;
}

std::string key_string(const CaseKey& k) {
    char buf[128];
    snprintf(buf, sizeof buf, "%dd %s%d %s %s %s c%d%s", k.ndim, k.shape == kStar ? "star" : "box",
             k.r, k.dtype == 0 ? "f32" : (k.dtype == 1 ? "f16" : "f64"), k.boundary == kPeriodic ? "periodic" : "zero",
             k.update == 0 ? "linear" : (k.update == 1 ? "wave" : (k.update == 2 ? "varcoef" : "wave-reverse")), k.size_class,
             k.slab == 0 ? "" : (k.slab == 1 ? " slab-few-planes" : (k.slab == 2 ? " slab-long-march" : " slab-across")));
    return buf;
}

static LaunchCfg default_cfg(const CaseKey& k) {
    LaunchCfg c{};
    if (k.update == kKeyWaveReverse) {
        // LDS-ring reverse kernel with 64 x 32 tiles (16 waves, one
        // workgroup per CU): measured best for the pointwise gradient step,
        // 43.0 against 44.6 ms with 64 x 16 tiles on the 256^3 x 200 case.
        c.variant = ST_VARIANT_WAVE3D_LDS;
        c.tile_y = 32;
        c.tsteps = 1;
        c.zchunk = kAutoChunk;
        return c;
    }
    if (k.update == ST_WAVE && k.dtype == 2) {
        // FP64 leapfrog: the z-march with queued partial sums; its radius-4
        // queue and weights take about 220 VGPRs at 2 rows per thread, so two
        // waves per SIMD, and 64 x 16 tiles of eight waves beat 64 x 8 tiles
        // of four (184 against 166 GCells/s on 512^3: a smaller halo share).
        c.variant = ST_VARIANT_WAVE3D;
        c.tile_y = 16;
        c.tsteps = 1;
        c.zchunk = kAutoChunk;
        return c;
    }
    if (k.update == ST_WAVE) {
        c.variant = ST_VARIANT_WAVE3D_LDS;
        c.tile_y = 32;
        c.tsteps = 1;
        c.zchunk = kAutoChunk;
        return c;
    }
    if (k.update == ST_VARCOEF) {
        c.variant = ST_VARIANT_VC3D;
        c.tile_y = k.shape == kStar && k.r == 1 ? 16 : 8;
        c.zchunk = kAutoChunk;
        return c;
    }
    if (k.ndim == 3) {
        c.variant = ST_VARIANT_ZM3D;
        c.tile_y = k.dtype == 0 ? 32 : 16;
        c.zchunk = kAutoChunk;
        // The 125-point box on a slab with few z planes marches y instead
        // (a march of a few planes computes partial sums for 2R planes
        // outside its chunk).
        if (k.shape == kBox && k.r == 2 && k.slab == 1) {
            c.variant = ST_VARIANT_YM3D;
            c.tile_y = 8;
        }
        return c;
    }
    if (k.size_class <= 1 && k.dtype != ST_F64) {   // (f64 in 2D: row march only)
        // Small grids: square LDS tiles give enough workgroups; deeper
        // fusion for narrow stencils (these launches are short).
        c.variant = ST_VARIANT_TB2D;
        c.tile_x = 64;
        c.tile_y = 32;
        c.tsteps = k.r == 1 ? 8 : (k.r == 2 ? 4 : 2);
        return c;
    }
    // Larger grids: the row march (redundant halo work in x only).
    c.variant = ST_VARIANT_YM2D;
    c.tile_x = 256;
    c.tile_y = 0;
    c.tsteps = k.r <= 2 ? 4 : 2;
    return c;
}

int varcoef_taps(const st_problem& p) {
    const int w = 2 * p.radius + 1;
    if (p.shape == ST_BOX) return p.ndim == 3 ? w * w * w : w * w;
    return 1 + 2 * p.ndim * p.radius;
}

// Starting configuration when a plan option forces a kernel family other
// than the map's: that family's own defaults (the other option fields then
// override them).
LaunchCfg variant_default(const st_problem& p, int variant) {
    const CaseKey k = classify(p);
    LaunchCfg c = default_cfg(k);
    if (variant == c.variant) return c;
    c = LaunchCfg{variant, 0, 0, 1, 0};
    switch (variant) {
        case ST_VARIANT_TB2D: c.tile_x = 64; c.tile_y = 32; c.tsteps = default_cfg(k).tsteps; break;
        case ST_VARIANT_YM2D: c.tile_x = 256; c.tile_y = 0; c.tsteps = default_cfg(k).tsteps; break;
        case ST_VARIANT_ZM3D: c.tile_y = 16; c.zchunk = kAutoChunk; break;
        case ST_VARIANT_ZM3D_MFMA: c.tile_y = 64; c.zchunk = kAutoChunk; break;
        case ST_VARIANT_ZM3D_H2: c.tile_y = 16; c.zchunk = kAutoChunk; break;
        case ST_VARIANT_YM3D: c.tile_y = 8; c.zchunk = kAutoChunk; break;
        case ST_VARIANT_YM2D_H2: c.tile_x = 256; c.tile_y = 0; c.tsteps = 2; break;
        case ST_VARIANT_WAVE3D: c.tile_y = 8; c.zchunk = kAutoChunk; break;
        case ST_VARIANT_WAVE3D_LDS: c.tile_y = 32; c.zchunk = kAutoChunk; break;
        default: break;
    }
    return c;
}

struct KeyLess {
    bool operator()(const CaseKey& a, const CaseKey& b) const {
        const int va[8] = {a.ndim, a.shape, a.r, a.dtype, a.boundary, a.update, a.size_class, a.slab};
        const int vb[8] = {b.ndim, b.shape, b.r, b.dtype, b.boundary, b.update, b.size_class, b.slab};
        return std::lexicographical_compare(va, va + 8, vb, vb + 8);
    }
};

static std::mutex g_map_mu;
static std::map<CaseKey, LaunchCfg, KeyLess> g_map;
static bool g_cache_loaded = false;

// Cache file format, one entry per line (later lines win):
//   ndim shape r dtype boundary update size_class slab variant tile_x tile_y tsteps zchunk
static void read_map_file(const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        CaseKey k;
        LaunchCfg c;
        if (sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d %d", &k.ndim, &k.shape, &k.r, &k.dtype,
                   &k.boundary, &k.update, &k.size_class, &k.slab, &c.variant, &c.tile_x,
                   &c.tile_y, &c.tsteps, &c.zchunk) == 13)
            g_map[k] = c;
    }
    fclose(f);
}

// The measured map shipped next to the library (written by the autotuner on
// an MI355X), then the caller's tuning cache on top of it.
static void load_cache_locked() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    Dl_info info;
    if (dladdr((void*)&read_map_file, &info) && info.dli_fname) {
        std::string dir(info.dli_fname);
        const size_t slash = dir.find_last_of('/');
        dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
        read_map_file((dir + "/dispatch_mi355x.txt").c_str());
    }
    const char* path = getenv("STENCIL_TUNE_CACHE");
    if (path && *path) read_map_file(path);
}

LaunchCfg default_dispatch(const CaseKey& k) { return default_cfg(k); }

LaunchCfg dispatch_lookup(const CaseKey& k) {
    std::lock_guard<std::mutex> lk(g_map_mu);
    load_cache_locked();
    auto it = g_map.find(k);
    if (it != g_map.end()) return it->second;
    return default_cfg(k);
}

void dispatch_store(const CaseKey& k, const LaunchCfg& c, bool persist) {
    std::lock_guard<std::mutex> lk(g_map_mu);
    load_cache_locked();
    g_map[k] = c;
    if (!persist) return;
    const char* path = getenv("STENCIL_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d\n", k.ndim, k.shape, k.r, k.dtype,
            k.boundary, k.update, k.size_class, k.slab, c.variant, c.tile_x, c.tile_y, c.tsteps,
            c.zchunk);
    fclose(f);
}

// Plane chunk giving about 1024 workgroups (four per CU) while keeping the
// z-halo re-read (2R planes per chunk) small; the measured map overrides it.
// Workgroups of a configuration that fit on one CU at once (register and
// LDS limits of the compiled kernels): the LDS-ring wave kernel runs 4-, 8-
// and 16-wave workgroups for 8-, 16- and 32-row tiles; the direct-form wave
// kernels (adjoint, gradient) hold about two waves per SIMD; the linear
// z-march runs four 4-wave workgroups.
static int resident_wgs(const st_problem& p, const LaunchCfg& c) {
    if (p.update == ST_WAVE && p.dtype == ST_F64) return c.tile_y >= 16 ? 1 : 2;   // 8- or 4-wave groups, 2 waves per SIMD
    if (p.update == ST_WAVE && c.variant == ST_VARIANT_WAVE3D_LDS)
        return c.tile_y >= 32 ? 1 : (c.tile_y >= 16 ? 2 : 3);
    if (p.update == ST_WAVE) return c.tile_y >= 32 ? 1 : 2;   // adjoint/gradient: ~2 waves per SIMD
    if (c.variant == ST_VARIANT_ZM3D_MFMA) return 2;
    if (c.variant == ST_VARIANT_VC3D) return 2;   // measured: fewer, longer marches stream best
    return 4;
}

static int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

// Plane chunk for a z-march: split z so that the grid fills every CU about
// once (one round of workgroups; a partial second round costs a whole
// round's time), with chunks of at least 16 planes.
int auto_zchunk(const st_problem& p0, const LaunchCfg& c, int resident) {
    st_problem p = p0;
    if (c.variant == ST_VARIANT_YM3D) {   // chunks of the y march over (x, z) tiles
        p.n[1] = p0.n[2];
        p.n[2] = p0.n[1];
    }
    const int rows = c.tile_y >= 64 ? 64 : (c.tile_y >= 32 ? 32 : (c.tile_y >= 16 ? 16 : 8));
    const int64_t tile_w = c.variant == ST_VARIANT_ZM3D_H2 ? 2 * kWave : kWave;   // H2: two cells per lane
    int64_t tiles = ((p.n[0] + tile_w - 1) / tile_w) * ((p.n[1] + rows - 1) / rows);
    if (p.update == ST_LINEAR && p.ndim == 3 && c.tsteps == 2)   // two-step tiles: 62 x (tile_y - 2) outputs
        tiles = ((p.n[0] + 61) / 62) * ((p.n[1] + rows - 3) / (rows - 2));
    const int64_t target = (int64_t)device_cus() * (resident > 0 ? resident : resident_wgs(p, c));
    const int64_t nch = (target + tiles - 1) / tiles;
    if (nch <= 1) return 0;
    int64_t zc = (p.n[2] + nch - 1) / nch;
    zc = zc < 16 ? 16 : zc;
    zc = (zc + 7) / 8 * 8;
    return zc >= p.n[2] ? 0 : (int)zc;
}

// The reverse step runs one step per launch in either wave kernel family.
bool adj_cfg_legal(const st_problem& p, const LaunchCfg& c) {
    return p.update == ST_WAVE && (c.variant == ST_VARIANT_WAVE3D_LDS || c.variant == ST_VARIANT_WAVE3D) &&
           (c.tile_y == 8 || c.tile_y == 16 || c.tile_y == 32) && c.zchunk >= 0 && c.tsteps >= 0 && c.tsteps <= 1;
}

bool cfg_legal(const st_problem& p, const LaunchCfg& c) {
    if (p.update == ST_WAVE && p.dtype == ST_F64)   // one FP64 kernel: 8- or 16-row tiles, one step
        return c.variant == ST_VARIANT_WAVE3D && (c.tile_y == 8 || c.tile_y == 16) && c.tile_x == 0 &&
               c.zchunk >= 0 && c.tsteps >= 0 && c.tsteps <= 1;
    if (p.update == ST_WAVE) {
        if (c.tsteps == 2 && !wave3d_tb2_supported(p.radius)) return false;
        if (c.variant == ST_VARIANT_WAVE3D_LDS)   // tile_x: planes staged per barrier (0 or 1: one, 2: two)
            return (c.tile_y == 8 || c.tile_y == 16 || c.tile_y == 32) && c.zchunk >= 0 && c.tsteps <= 1 &&
                   c.tile_x >= 0 && c.tile_x <= 2;
        return c.variant == ST_VARIANT_WAVE3D && (c.tile_y == 8 || c.tile_y == 16 || c.tile_y == 32) &&
               c.zchunk >= 0 && c.tsteps >= 0 && c.tsteps <= 2;
    }
    if (p.update == ST_VARCOEF)
        return c.variant == ST_VARIANT_VC3D && (c.tile_y == 8 || (c.tile_y == 16 && p.shape == ST_STAR && p.radius == 1)) &&
               c.zchunk >= 0 && c.tsteps >= 0 && c.tsteps <= 1;
    if (p.ndim == 3) {
        if (c.variant == ST_VARIANT_ZM3D_MFMA)
            return p.shape == ST_BOX && p.radius == 1 && p.dtype == ST_F16 && p.n[0] % 8 == 0 &&
                   c.tile_y == 64 && c.zchunk >= 0;
        if (c.variant == ST_VARIANT_YM3D) {
            const size_t esz = p.dtype == ST_F16 ? 2 : (p.dtype == ST_F64 ? 8 : 4);
            return p.shape == ST_BOX && p.radius <= 2 &&
                   (size_t)p.n[0] * p.n[1] * p.n[2] * esz <= 0xFFFFFFFFull &&
                   (c.tile_y == 8 || c.tile_y == 16 || (c.tile_y == 32 && p.dtype != ST_F64)) && c.zchunk >= 0 &&
                   c.tsteps >= 0 && c.tsteps <= 1;
        }
        if (c.variant == ST_VARIANT_ZM3D_H2)
            return (p.shape == ST_BOX ? p.radius <= 2 : p.radius == 1) && p.dtype == ST_F16 && p.n[0] % 2 == 0 &&
                   (c.tile_y == 8 || c.tile_y == 16 || c.tile_y == 32) && c.zchunk >= 0 && c.tsteps <= 1;
        if (c.variant == ST_VARIANT_ZM3D && c.tsteps == 2 &&
            (!zm3d_tb2_supported(p.radius, p.shape) || (c.tile_y != 16 && c.tile_y != 32)))
            return false;
        if (p.dtype == ST_F64)   // f64: one step per launch, 8- or 16-row tiles
            return c.variant == ST_VARIANT_ZM3D && (c.tile_y == 8 || c.tile_y == 16) && c.zchunk >= 0 &&
                   c.tsteps >= 0 && c.tsteps <= 1;
        return c.variant == ST_VARIANT_ZM3D && (c.tile_y == 8 || c.tile_y == 16 || c.tile_y == 32) &&
               c.zchunk >= 0 && c.tsteps >= 0 && c.tsteps <= 2;
    }
    if (c.variant == ST_VARIANT_YM2D_H2) {
        if (p.shape != ST_BOX || p.radius > 2 || p.dtype != ST_F16 || p.n[0] % 2 != 0) return false;
        if (c.tile_x != 256 && c.tile_x != 512) return false;
        if (c.tile_y < 0 || c.tsteps < 1 || c.tsteps > 16 || c.tile_x - 2 * c.tsteps < kWave) return false;
        return ym2d_h2_lds_bytes(c.tile_x, c.tsteps, p.radius) <= ym2d_max_lds_bytes();
    }
    if (c.variant == ST_VARIANT_YM2D) {
        if (c.tile_x != 256 && c.tile_x != 512) return false;
        if (c.tile_y < 0 || c.tsteps < 1 || c.tsteps > 16) return false;
        if (c.tile_x - 2 * c.tsteps * p.radius < kWave) return false;
        return ym2d_lds_bytes(c.tile_x, c.tsteps, p.radius, p.dtype == ST_F64 ? 8 : 4) <= ym2d_max_lds_bytes();
    }
    if (c.variant != ST_VARIANT_TB2D || p.dtype == ST_F64) return false;
    // zchunk: waves per workgroup (0 = 4).
    if (c.zchunk != 0 && c.zchunk != 4 && c.zchunk != 8 && c.zchunk != 16) return false;
    if (c.tile_x < 8 || c.tile_x > 512) return false;
    if (c.tile_y < 4 || c.tile_y > 512 || c.tsteps < 1 || c.tsteps > 16) return false;
    return (int)sizeof(float) * tb2d_lds_floats_host(c.tile_x, c.tile_y, c.tsteps, p.radius) <=
           tb2d_max_lds_bytes();
}

}  // namespace stk
