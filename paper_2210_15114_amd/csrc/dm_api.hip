// dm_api.hip - the C ABI (include/dm.h): argument validation, workspace
// layout, the handle, and the order of kernel launches for preparation
// (Algorithm 1) and queries (Algorithms 2 and 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/dm.h"
#include "dm_internal.h"

using namespace dm;

namespace {

constexpr size_t ALIGN = 256;
inline size_t al(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

bool valid_metric(int32_t m) { return m >= DM_L1 && m <= DM_BILINEAR; }
// the power p of f(x, y) = sum_k |x(k) - y(k)|^p (TV: p = 1, halved; the
// divergences and quadratic forms: 1, unused)
int metric_power(int32_t m) {
    switch (m) {
    case DM_L2SQ: return 2;
    case DM_L3: return 3;
    case DM_L4: return 4;
    case DM_L5: return 5;
    case DM_L6: return 6;
    default: return 1;
    }
}
// metrics answered by moments and one pass over the points (Appendix A)
bool sf_metric(int32_t m) { return m >= DM_L4 && m <= DM_BILINEAR; }
int sf_form(int32_t m) {
    if (m == DM_L4 || m == DM_L6) return SF_EVEN;
    if (m == DM_KL || m == DM_CE) return SF_LOG;
    return SF_LIN;
}
// metrics whose definition carries a d x d matrix (dm_prepare_matrix)
bool matrix_metric(int32_t m) { return m == DM_MAHA2 || m == DM_BILINEAR; }
// metrics defined on float data only
bool float_only_metric(int32_t m) { return m == DM_TV || m == DM_KL || m == DM_CE || matrix_metric(m); }
// metrics answered by the l1 pass (TV is half the l1 distance)
bool l1_pass_metric(int32_t m) { return m == DM_L1 || m == DM_TV; }
// odd p >= 3: the sorted path with p + 1 running sums
bool lp_metric(int32_t m) { return m == DM_L3 || m == DM_L5; }
// metrics that sort the coordinates at preparation (Algorithm 1)
bool sorted_metric(int32_t m) { return l1_pass_metric(m) || lp_metric(m); }
bool valid_dtype(int32_t t) { return t == DM_F32 || t == DM_F64 || t == DM_I32 || t == DM_I64; }
bool int_dtype(int32_t t) { return t == DM_I32 || t == DM_I64; }
size_t dtype_size(int32_t t) { return (t == DM_F64 || t == DM_I64) ? 8 : 4; }

constexpr int32_t L2_MAX_D = 512;   // LDS staging bound of the l2-squared kernels

// Control block owned by a handle: sticky status, chained-scan state, totals.
struct Ctl {
    uint32_t status;
    uint32_t pad[63];
    ChainState chain;
    double T0[1024];
    double U[1024];
    double zl1[1024];
};

// A look-back record region of one pass kernel shape (its ticket class).
struct RegionSpec {
    int cls;
    size_t off;     // byte offset in the workspace
    size_t words;   // 64-bit words
};

// Byte layout of one dataset's workspace: the preparation results, the sort's
// temporaries and everything a query needs (control block, scratch for
// b <= MAX_B, the record regions of every pass shape the handle can launch,
// the single-column group buffer), so that a caller who passes the workspace
// owns all device memory the handle uses.
struct Layout {
    int64_t ld = 0;         // stride between coordinates of the d x n arrays
    uint32_t ntiles = 0;    // sort tiles
    size_t perm = 0, xs = 0, ids = 0, rowsum = 0, rownrm = 0, xcopy = 0, kmin = 0, kmax = 0, flags = 0;
    size_t centre = 0, mat = 0;   // per-coordinate centre (FP64); M and W (d x d each) of the quadratic forms
    size_t c32 = 0;               // per-coordinate FP32 centre of the sorted metrics and l2 squared
    size_t logx = 0;              // FP64 logarithms of the points (KL divergence, cross entropy)
    size_t key_off = 0, key_len = 0, tile_off = 0, tile_seg = 0;
    size_t k1 = 0, v1 = 0, counts = 0;
    size_t ctl = 0;                       // Ctl
    size_t qscratch = 0, qscratch_bytes = 0;   // query scratch (totals partials, moments, l2 partials)
    size_t single = 0, single_bytes = 0;  // single-column group buffer (l1, TV)
    int32_t single_group = 0;             // coordinates per group of that buffer
    size_t regions_begin = 0, regions_end = 0;
    std::vector<RegionSpec> regions;
    size_t total = 0;
};

constexpr int32_t MAX_B = 64;

size_t query_scratch_bytes(int64_t n, int32_t d, int32_t metric, int32_t b) {
    size_t s = al(totals_scratch_bytes(n, b));
    if (metric == DM_L2SQ) s += al(l2_scratch_bytes(n, d, b));
    if (sf_metric(metric)) s += al(sf_scratch_bytes(n, d, b, sf_form(metric), metric_power(metric)));
    if (lp_metric(metric)) s += al(lp_moments_bytes(n, d, b, metric_power(metric)));
    return s;
}

int kind_index(bool is_int, int zkind) { return !is_int ? 0 : zkind == IN_I32 ? 1 : 2; }

int log2_pad(int32_t b) {
    int lg = 0;
    while ((1 << lg) < b) ++lg;
    return lg;
}

// the ticket class and record region size of an odd-p pass
L1Shape lp_shape_of(int64_t n, int p, bool is_int, int32_t b, int zkind) {
    L1Shape sh;
    sh.cls = L1_CLASSES + (kind_index(is_int, zkind) * 8 + log2_pad(b)) * 2 + (p == 5 ? 1 : 0);
    sh.record_words = lp_record_words(n, b, is_int, p);
    return sh;
}

// Coordinates per group of a single-column l1 query (group x ld values of
// FP32 or int64 in the buffer).
int32_t single_group_of(int64_t ld, int32_t d, bool is_int) {
    const size_t per = (size_t)ld * (is_int ? 8 : 4);
    const size_t g = SINGLE_GROUP_BYTES / per;
    return (int32_t)(g < 1 ? 1 : g > (size_t)d ? (size_t)d : g);
}

Layout make_layout(int64_t n, int32_t d, int32_t metric, int32_t dtype) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += al(bytes);
        return at;
    };
    L.ld = (n + 63) / 64 * 64;
    const size_t arr = (size_t)d * (size_t)L.ld * 4;
    if (sorted_metric(metric)) {
        L.ntiles = (uint32_t)((size_t)d * (size_t)((n + SORT_TILE - 1) / SORT_TILE));
        L.perm = take(arr);
        L.xs = take(arr);
        L.ids = take(arr);   // point ids of the middle sort passes
    }
    // a row-major FP32 / int32 copy of X: for the l2-squared products and for
    // the per-coordinate moments of odd p
    if (!sorted_metric(metric) || lp_metric(metric)) L.xcopy = take((size_t)n * d * 4);
    L.rowsum = take((size_t)n * 8);
    L.rownrm = take((size_t)n * 8);
    L.kmin = take((size_t)d * 4);
    L.kmax = take((size_t)d * 4);
    L.flags = take(16);
    L.centre = take((size_t)d * 8);
    L.c32 = take((size_t)d * 4);
    if (matrix_metric(metric)) L.mat = take((size_t)d * d * 16);
    if (metric == DM_KL || metric == DM_CE) L.logx = take((size_t)n * d * 8);
    if (sorted_metric(metric)) {
        L.key_off = take((size_t)d * 8);
        L.key_len = take((size_t)d * 8);
        L.tile_off = take((size_t)(d + 1) * 4);
        L.tile_seg = take((size_t)L.ntiles * 4);
        L.k1 = take(arr);
        L.v1 = take(arr);
        L.counts = take((size_t)L.ntiles * 256 * 4);
    }
    // ---- what queries use ----
    const bool is_int = int_dtype(dtype);
    L.ctl = take(sizeof(Ctl));
    for (int32_t b = 1; b <= MAX_B; ++b) L.qscratch_bytes = std::max(L.qscratch_bytes, query_scratch_bytes(n, d, metric, b));
    L.qscratch = take(L.qscratch_bytes);
    if (l1_pass_metric(metric)) {
        L.single_group = single_group_of(L.ld, d, is_int);
        L.single_bytes = (size_t)L.single_group * (size_t)L.ld * (is_int ? 8 : 4);
        L.single = take(L.single_bytes);
    }
    // record regions of every pass shape reachable with b <= MAX_B, any tile
    // variant and (integer data) either right-hand-side type
    L.regions_begin = o;
    auto region = [&](const L1Shape& sh) {
        for (auto& r : L.regions)
            if (r.cls == sh.cls) return;
        L.regions.push_back(RegionSpec{sh.cls, take(sh.record_words * 8), sh.record_words});
    };
    const int kinds[2] = {is_int ? IN_I32 : IN_F32, IN_I64};
    for (int ki = 0; ki < (is_int ? 2 : 1); ++ki)
        for (int32_t bp = 1; bp <= MAX_B; bp <<= 1) {
            if (l1_pass_metric(metric)) {
                for (int v = 0; v < L1_VARIANTS; ++v) {
                    region(l1_shape(n, bp, is_int, kinds[ki], v));
                    if (bp == 1) region(l1_single_shape(n, is_int, kinds[ki], v));
                }
            } else if (lp_metric(metric)) {
                region(lp_shape_of(n, metric_power(metric), is_int, bp, kinds[ki]));
            }
        }
    L.regions_end = o;
    L.total = o;
    return L;
}

dm_status check_shape(int64_t n, int32_t d, int32_t metric, int32_t dtype) {
    if (n < 1 || d < 1) return DM_ERR_ARG;
    if (!valid_metric(metric) || !valid_dtype(dtype)) return DM_ERR_ARG;
    const int64_t ld = (n + 63) / 64 * 64;
    if ((uint64_t)ld * (uint64_t)d >= (1ull << 32)) return DM_ERR_ARG;   // 32-bit positions
    if (metric == DM_L2SQ && d > L2_MAX_D) return DM_ERR_ARG;
    if (float_only_metric(metric) && int_dtype(dtype)) return DM_ERR_DTYPE;
    if ((uint64_t)d * (uint64_t)d * 16 >= (1ull << 40)) return DM_ERR_ARG;
    return DM_OK;
}

dm_status from_hip(hipError_t e) {
    if (e == hipSuccess) return DM_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DM_ERR_NOMEM;
    return DM_ERR_DEVICE;
}

#define DM_TRY(expr)                         \
    do {                                     \
        hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) return from_hip(e_); \
    } while (0)

dm_status device_ready(int* dev) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return DM_ERR_DEVICE;
    if (hipGetDevice(dev) != hipSuccess) return DM_ERR_DEVICE;
    return DM_OK;
}

}  // namespace

struct MultiState;

struct dm_handle {
    MultiState* multi = nullptr;   // non-NULL for a multi-dataset handle
    int device = 0;
    int64_t n = 0;
    int32_t d = 0;
    int32_t metric = 0;
    int32_t dtype = 0;
    bool is_int = false;
    Layout L;
    char* ws = nullptr;
    bool owns_ws = false;
    Ctl* ctl = nullptr;   // in the workspace
    double guard_scale = 0.0;   // sum over the coordinates of range^p
    bool symmetric = true;      // A = A^T (false for the divergences and a non-symmetric bilinear form)
    hipStream_t last = nullptr;
    // Captured queries: dm_matvec records a query's launches once per
    // (Z, Out, b, right-hand-side type) in a hipGraph on a private capture
    // stream and replays it afterwards (least recently used of GRAPHS kept).
    struct Graph { const void* Z; void* Out; int32_t b; int zkind; hipGraphExec_t exec; uint64_t used; };
    static constexpr int GRAPHS = 4;
    std::vector<Graph> graphs;
    uint64_t graph_clock = 0;
    hipStream_t cap = nullptr;
    bool use_graphs = true;
    // tile variant of the l1 pass per (data path, log2 of the padded block
    // width); -1 until set, tuned or found in the tuning cache (then 0)
    int8_t variant[3][8];
    char arch[64] = {0};

    // measurement: event pairs around launches while profiling is on
    struct Ev { hipEvent_t a = nullptr, b = nullptr; int cls = 0; };
    bool prof = false;
    std::vector<Ev> evs;
    size_t ev_used = 0;
    double prof_ms[DM_K_CLASSES] = {0, 0, 0};
    int64_t prof_n[DM_K_CLASSES] = {0, 0, 0};

    template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

void release_multi(MultiState* m);

void drop_graphs(dm_handle* h) {
    for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

void release(dm_handle* h) {
    if (!h) return;
    if (h->multi) release_multi(h->multi);
    if (!h->graphs.empty() && h->last) (void)hipStreamSynchronize(h->last);
    drop_graphs(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (auto& e : h->evs) {
        if (e.a) (void)hipEventDestroy(e.a);
        if (e.b) (void)hipEventDestroy(e.b);
    }
    if (h->owns_ws && h->ws) (void)hipFree(h->ws);
    delete h;
}

void arch_name(int dev, char* out) {
    hipDeviceProp_t p;
    size_t i = 0;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
        // the base name only ("gfx950:sramecc+:xnack-" -> "gfx950")
        for (; i < 63 && p.gcnArchName[i] && p.gcnArchName[i] != ':'; ++i) out[i] = p.gcnArchName[i];
    }
    out[i] = 0;
}

int floor_log2(int64_t n) {
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= n) ++lg;
    return lg;
}
// the pass data path of a right-hand-side type on this handle
dm_status zkind_of(const dm_handle* h, int32_t z_dtype, int* zkind) {
    if (!valid_dtype(z_dtype)) return DM_ERR_ARG;
    if (h->is_int ? !(z_dtype == DM_I32 || z_dtype == DM_I64) : z_dtype != DM_F32) return DM_ERR_DTYPE;
    *zkind = h->is_int ? (z_dtype == DM_I32 ? IN_I32 : IN_I64) : IN_F32;
    return DM_OK;
}

// Tuning cache: the text file named by DM_TUNE_CACHE, one line per tuned
// configuration,
//   dmtune1 <arch> <metric> <dtype> <data path> <floor log2 n> <d> <log2 padded b> <variant>
// appended by dm_tune and read when a handle first needs the variant of a
// configuration; the last matching line wins.
int cache_lookup(const dm_handle* h, int kind, int lg) {
    const char* path = std::getenv("DM_TUNE_CACHE");
    if (!path || !*path || !h->arch[0]) return -1;
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    char line[256];
    int found = -1;
    while (std::fgets(line, sizeof line, f)) {
        char tag[16], arch[64];
        int metric, dtype, k, lgn, d, l, v;
        if (std::sscanf(line, "%15s %63s %d %d %d %d %d %d %d", tag, arch, &metric, &dtype, &k, &lgn, &d, &l, &v) != 9)
            continue;
        if (std::strcmp(tag, "dmtune1") != 0 || std::strcmp(arch, h->arch) != 0) continue;
        if (metric == h->metric && dtype == h->dtype && k == kind && lgn == floor_log2(h->n) && d == h->d &&
            l == lg && v >= 0 && v < L1_VARIANTS)
            found = v;
    }
    std::fclose(f);
    return found;
}

void cache_store(const dm_handle* h, int kind, int lg, int v) {
    const char* path = std::getenv("DM_TUNE_CACHE");
    if (!path || !*path || !h->arch[0]) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "dmtune1 %s %d %d %d %d %d %d %d\n", h->arch, h->metric, h->dtype, kind, floor_log2(h->n), h->d,
                 lg, v);
    std::fclose(f);
}

// the tile variant used for (data path, padded block width): set, tuned,
// cached, or the default
int variant_for(dm_handle* h, int kind, int lg) {
    int8_t& v = h->variant[kind][lg];
    if (v < 0) {
        const int c = cache_lookup(h, kind, lg);
        v = (int8_t)(c >= 0 ? c : 0);
    }
    return v;
}

double key_to_double(uint32_t k, bool is_int) {
    if (is_int) return (double)(int32_t)(k ^ 0x80000000u);
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

// the ticket class and record region size of an odd-p pass
L1Shape lp_shape(const dm_handle* h, int32_t b, int zkind) {
    return lp_shape_of(h->n, metric_power(h->metric), h->is_int, b, zkind);
}

// the record region of one pass shape (carved from the workspace at
// preparation and zeroed there)
dm_status region_for(dm_handle* h, const L1Shape& sh, uint64_t** out) {
    for (auto& r : h->L.regions)
        if (r.cls == sh.cls && r.words >= sh.record_words) {
            *out = h->at<uint64_t>(r.off);
            return DM_OK;
        }
    return DM_ERR_STATE;   // not a shape this handle was laid out for
}

// Bracket one launch with events when profiling is on.
struct ProfScope {
    dm_handle* h;
    dm_handle::Ev* ev = nullptr;
    hipStream_t s;
    ProfScope(dm_handle* hh, int cls, hipStream_t ss) : h(hh), s(ss) {
        if (!h->prof) return;
        if (h->ev_used == h->evs.size()) {
            dm_handle::Ev e;
            if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) return;
            h->evs.push_back(e);
        }
        ev = &h->evs[h->ev_used++];
        ev->cls = cls;
        (void)hipEventRecord(ev->a, s);
    }
    ~ProfScope() {
        if (ev) (void)hipEventRecord(ev->b, s);
    }
};

dm_status prepare_l1(dm_handle* h, const void* X, hipStream_t s) {
    const Layout& L = h->L;
    const int64_t n = h->n;
    const int32_t d = h->d;
    // segment tables: coordinate k is segment k
    const uint32_t tps = (uint32_t)((n + SORT_TILE - 1) / SORT_TILE);
    std::vector<int64_t> koff(d), klen(d, n);
    std::vector<uint32_t> toff(d + 1), tseg((size_t)L.ntiles);
    for (int32_t k = 0; k < d; ++k) {
        koff[k] = (int64_t)k * L.ld;
        toff[k] = (uint32_t)k * tps;
        for (uint32_t t = 0; t < tps; ++t) tseg[(size_t)k * tps + t] = (uint32_t)k;
    }
    toff[d] = (uint32_t)d * tps;
    DM_TRY(hipMemcpyAsync(h->ws + L.key_off, koff.data(), koff.size() * 8, hipMemcpyHostToDevice, s));
    DM_TRY(hipMemcpyAsync(h->ws + L.key_len, klen.data(), klen.size() * 8, hipMemcpyHostToDevice, s));
    DM_TRY(hipMemcpyAsync(h->ws + L.tile_off, toff.data(), toff.size() * 4, hipMemcpyHostToDevice, s));
    DM_TRY(hipMemcpyAsync(h->ws + L.tile_seg, tseg.data(), tseg.size() * 4, hipMemcpyHostToDevice, s));
    DM_TRY(hipStreamSynchronize(s));   // the host vectors die with this frame

    SegTables tb;
    tb.key_off = h->at<int64_t>(L.key_off);
    tb.key_len = h->at<int64_t>(L.key_len);
    tb.tile_off = h->at<uint32_t>(L.tile_off);
    tb.tile_seg = h->at<uint32_t>(L.tile_seg);
    tb.seg_int = nullptr;
    tb.centre = h->is_int ? nullptr : h->at<float>(L.c32);
    tb.nseg = d;
    tb.ntiles = L.ntiles;

    uint32_t* K0 = h->at<uint32_t>(L.xs);     // keys after transposition; becomes xs
    uint32_t* V0 = h->at<uint32_t>(L.ids);   // point ids after pass 2
    uint32_t* K1 = h->at<uint32_t>(L.k1);
    uint32_t* V1 = h->at<uint32_t>(L.v1);
    uint32_t* perm = h->at<uint32_t>(L.perm);
    uint32_t* counts = h->at<uint32_t>(L.counts);

    DM_TRY(launch_prep_transpose(h->dtype, X, n, d, K0, L.ld, nullptr, h->at<uint32_t>(L.kmin),
                                 h->at<uint32_t>(L.kmax), h->at<uint32_t>(L.flags), s));
    // float coordinates are shifted by their centres (exact) before anything
    // is formed from them: sorted values, row statistics, the point copy
    if (!h->is_int) DM_TRY(launch_centre(h->at<uint32_t>(L.kmin), h->at<uint32_t>(L.kmax), d, h->at<float>(L.c32), s));
    DM_TRY(launch_row_stats(h->dtype, X, n, d, h->ws + L.rowsum, h->ws + L.rownrm, s, metric_power(h->metric),
                            tb.centre, lp_metric(h->metric) ? h->ws + L.xcopy : nullptr));

    const uint32_t* kin[4] = {K0, K1, K0, K1};
    const uint32_t* vin[4] = {nullptr, V1, V0, V1};
    uint32_t* kout[4] = {K1, K0, K1, K0};
    uint32_t* vout[4] = {V1, V0, V1, perm};
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        DM_TRY(launch_sort_count(kin[pass], counts, tb, shift, s));
        DM_TRY(launch_sort_scan(counts, tb, s));
        DM_TRY(launch_sort_scatter(kin[pass], vin[pass], kout[pass], vout[pass], counts, tb, shift, pass == 0,
                                   pass == 3, h->is_int, s));
    }
    return DM_OK;
}

// The sort-free metrics (Appendix A): the per-coordinate centre, the domain
// check and per-point weights of the divergences, and the matrices of the
// quadratic forms.  Blocking.
dm_status prepare_sortfree(dm_handle* h, const std::vector<uint32_t>& kmin, const std::vector<uint32_t>& kmax,
                           const double* M, hipStream_t s) {
    const int32_t d = h->d;
    const int64_t n = h->n;
    const Layout& L = h->L;
    // centre c_k = midpoint of the coordinate's range (integer data: rounded
    // down, so the centred values stay integers); the even-p and Mahalanobis
    // moments of x - c are bounded by the range instead of the magnitude
    if (h->is_int) {
        std::vector<int64_t> c(d);
        for (int32_t k = 0; k < d; ++k) {
            const int64_t lo = (int32_t)(kmin[k] ^ 0x80000000u), hi = (int32_t)(kmax[k] ^ 0x80000000u);
            c[k] = (lo + hi) >> 1;
        }
        DM_TRY(hipMemcpy(h->ws + L.centre, c.data(), (size_t)d * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<double> c(d);
        for (int32_t k = 0; k < d; ++k) c[k] = 0.5 * (key_to_double(kmin[k], false) + key_to_double(kmax[k], false));
        DM_TRY(hipMemcpy(h->ws + L.centre, c.data(), (size_t)d * 8, hipMemcpyHostToDevice));
    }
    const float* xc = h->at<float>(L.xcopy);
    if (h->metric == DM_KL || h->metric == DM_CE) {
        h->symmetric = false;
        DM_TRY(launch_fill_u32(h->at<uint32_t>(L.flags), 0u, 4, s));
        DM_TRY(launch_kl_weights(xc, n, d, h->at<double>(L.rowsum), h->at<double>(L.logx), h->at<uint32_t>(L.flags),
                                 FLAG_DOMAIN, s));
        DM_TRY(hipStreamSynchronize(s));
        uint32_t f = 0;
        DM_TRY(hipMemcpy(&f, h->ws + L.flags, 4, hipMemcpyDeviceToHost));
        if (f & FLAG_DOMAIN) return DM_ERR_ARG;
    }
    if (matrix_metric(h->metric)) {
        const size_t dd = (size_t)d * d;
        std::vector<double> mw(2 * dd);
        for (size_t e = 0; e < dd; ++e) {
            if (!std::isfinite(M[e])) return DM_ERR_NONFINITE;
            mw[e] = M[e];
        }
        for (int32_t k = 0; k < d; ++k)
            for (int32_t l = 0; l < d; ++l) {
                const double mkl = M[(size_t)k * d + l], mlk = M[(size_t)l * d + k];
                // Mahalanobis: sum_j z_j (x_i - x_j)^T M (x_i - x_j) carries
                // -x_i^T (M + M^T) sum_j z_j x_j; the bilinear form carries M
                mw[dd + (size_t)k * d + l] = h->metric == DM_MAHA2 ? -(mkl + mlk) : mkl;
                if (h->metric == DM_BILINEAR && mkl != mlk) h->symmetric = false;
            }
        DM_TRY(hipMemcpy(h->ws + L.mat, mw.data(), 2 * dd * 8, hipMemcpyHostToDevice));
        if (h->metric == DM_MAHA2)
            DM_TRY(launch_maha_weights(xc, h->at<double>(L.centre), n, d, h->at<double>(L.mat), h->at<double>(L.rowsum),
                                       s));
        DM_TRY(hipStreamSynchronize(s));
    }
    return DM_OK;
}

}  // namespace

extern "C" {

const char* dm_status_string(int32_t status) {
    switch (status) {
    case DM_OK: return "ok";
    case DM_ERR_ARG: return "invalid argument";
    case DM_ERR_NONFINITE: return "non-finite value (NaN or Inf)";
    case DM_ERR_OVERFLOW: return "integer result may exceed int64";
    case DM_ERR_NOMEM: return "device memory allocation failed";
    case DM_ERR_DEVICE: return "no usable HIP device or a HIP call failed";
    case DM_ERR_DTYPE: return "dtype not allowed here (or integer |x| >= 2^31)";
    case DM_ERR_STATE: return "operation not supported by this handle";
    default: return "unknown status";
    }
}

dm_status dm_workspace_size(int64_t n, int32_t d, int32_t metric, int32_t dtype, size_t* bytes) {
    if (!bytes) return DM_ERR_ARG;
    dm_status st = check_shape(n, d, metric, dtype);
    if (st != DM_OK) return st;
    *bytes = make_layout(n, d, metric, dtype).total;
    return DM_OK;
}

int dm_int_bound_ok(double sum_ranges, double z_l1) {
    if (!(sum_ranges >= 0.0) || !(z_l1 >= 0.0)) return 0;
    return (z_l1 * sum_ranges < 4611686018427387904.0) ? 1 : 0;   // 2^62
}

static dm_status prepare_impl(const void* X, int64_t n, int32_t d, int32_t metric, int32_t dtype, const double* M,
                              void* workspace, size_t ws_bytes, void* stream, dm_handle** out) {
    if (!out) return DM_ERR_ARG;
    *out = nullptr;
    if (!X) return DM_ERR_ARG;
    dm_status st = check_shape(n, d, metric, dtype);
    if (st != DM_OK) return st;
    const Layout L = make_layout(n, d, metric, dtype);
    if (workspace && ws_bytes < L.total) return DM_ERR_ARG;
    if (workspace && ((uintptr_t)workspace % ALIGN) != 0) return DM_ERR_ARG;
    int dev = 0;
    if ((st = device_ready(&dev)) != DM_OK) return st;

    hipStream_t s = (hipStream_t)stream;
    dm_handle* h = new (std::nothrow) dm_handle();
    if (!h) return DM_ERR_NOMEM;
    h->device = dev;
    h->n = n;
    h->d = d;
    h->metric = metric;
    h->dtype = dtype;
    h->is_int = int_dtype(dtype);
    h->L = L;
    std::memset(h->variant, -1, sizeof h->variant);
    arch_name(dev, h->arch);
    {   // DM_QUERY_GRAPH=0: launch every query eagerly instead of replaying graphs
        const char* e = std::getenv("DM_QUERY_GRAPH");
        h->use_graphs = !(e && e[0] == '0');
    }
    auto fail = [&](dm_status e) {
        release(h);
        return e;
    };
    if (workspace) {
        h->ws = (char*)workspace;
    } else {
        void* p = nullptr;
        if (hipMalloc(&p, L.total) != hipSuccess) return fail(DM_ERR_NOMEM);
        h->ws = (char*)p;
        h->owns_ws = true;
    }
    h->ctl = h->at<Ctl>(L.ctl);
    Ctl init;
    std::memset(&init, 0, sizeof(init));
    if (hipMemcpyAsync(h->ctl, &init, sizeof(Ctl), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(DM_ERR_DEVICE);
    // query scratch and the look-back record regions start at zero (a zero
    // word carries no pass tag)
    if (launch_fill_u32(h->at<uint32_t>(L.qscratch), 0u, L.qscratch_bytes / 4, s) != hipSuccess ||
        launch_fill_u32(h->at<uint32_t>(L.regions_begin), 0u, (L.regions_end - L.regions_begin) / 4, s) !=
            hipSuccess)
        return fail(DM_ERR_DEVICE);
    if (launch_fill_u32(h->at<uint32_t>(L.kmin), 0xffffffffu, (size_t)d, s) != hipSuccess ||
        launch_fill_u32(h->at<uint32_t>(L.kmax), 0u, (size_t)d, s) != hipSuccess ||
        launch_fill_u32(h->at<uint32_t>(L.flags), 0u, 4, s) != hipSuccess)
        return fail(DM_ERR_DEVICE);

    if (sorted_metric(metric)) {
        if ((st = prepare_l1(h, X, s)) != DM_OK) return fail(st);
    } else if (metric == DM_L2SQ) {
        // the point copy, squared norms and (float data) centres as for the
        // sorted metrics; the l2-squared query sees only centred points
        const float* c = h->is_int ? nullptr : h->at<float>(L.c32);
        if (launch_prep_transpose(dtype, X, n, d, nullptr, 0, nullptr, h->at<uint32_t>(L.kmin),
                                  h->at<uint32_t>(L.kmax), h->at<uint32_t>(L.flags), s) != hipSuccess ||
            (c && launch_centre(h->at<uint32_t>(L.kmin), h->at<uint32_t>(L.kmax), d, h->at<float>(L.c32), s) !=
                      hipSuccess) ||
            launch_row_stats(dtype, X, n, d, h->ws + L.rowsum, h->ws + L.rownrm, s, 1, c, h->ws + L.xcopy) !=
                hipSuccess)
            return fail(DM_ERR_DEVICE);
    } else {
        // the sort-free metrics keep the raw point copy (they centre in FP64 at use)
        if (launch_prep_transpose(dtype, X, n, d, nullptr, 0, h->ws + L.xcopy, h->at<uint32_t>(L.kmin),
                                  h->at<uint32_t>(L.kmax), h->at<uint32_t>(L.flags), s) != hipSuccess)
            return fail(DM_ERR_DEVICE);
        if (launch_row_stats(dtype, X, n, d, h->ws + L.rowsum, h->ws + L.rownrm, s) != hipSuccess)
            return fail(DM_ERR_DEVICE);
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(DM_ERR_DEVICE);
    uint32_t flags = 0;
    std::vector<uint32_t> kmin(d), kmax(d);
    if (hipMemcpy(&flags, h->ws + L.flags, 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(kmin.data(), h->ws + L.kmin, (size_t)d * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(kmax.data(), h->ws + L.kmax, (size_t)d * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(DM_ERR_DEVICE);
    if (flags & FLAG_NONFINITE) return fail(DM_ERR_NONFINITE);
    if (flags & FLAG_INT_RANGE) return fail(DM_ERR_DTYPE);
    double g = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        const double r = key_to_double(kmax[k], h->is_int) - key_to_double(kmin[k], h->is_int);
        double rp = r;
        for (int e = 1; e < metric_power(metric); ++e) rp *= r;
        g += rp;
    }
    h->guard_scale = g;
    if (sf_metric(metric) && (st = prepare_sortfree(h, kmin, kmax, M, s)) != DM_OK) return fail(st);
    h->last = s;
    *out = h;
    return DM_OK;
}

dm_status dm_prepare(const void* X, int64_t n, int32_t d, int32_t metric, int32_t dtype, void* workspace,
                     size_t ws_bytes, void* stream, dm_handle** out) {
    if (matrix_metric(metric)) {
        if (out) *out = nullptr;
        return DM_ERR_ARG;   // the quadratic forms need their matrix: dm_prepare_matrix
    }
    return prepare_impl(X, n, d, metric, dtype, nullptr, workspace, ws_bytes, stream, out);
}

dm_status dm_prepare_matrix(const void* X, int64_t n, int32_t d, int32_t metric, int32_t dtype, const double* M,
                            void* workspace, size_t ws_bytes, void* stream, dm_handle** out) {
    if (!matrix_metric(metric) || !M) {
        if (out) *out = nullptr;
        return DM_ERR_ARG;
    }
    return prepare_impl(X, n, d, metric, dtype, M, workspace, ws_bytes, stream, out);
}

dm_status dm_reserve(dm_handle* h, int32_t b) {
    if (!h || b < 1 || b > MAX_B) return DM_ERR_ARG;
    if (h->multi) return DM_ERR_STATE;
    return DM_OK;   // the workspace already holds what any query needs
}

}  // extern "C"

namespace {

// Where a query's scratch lives: the handle's workspace (dm_matvec) or the
// library's static device array (dm_matvec_static).
struct QueryMem {
    char* scratch = nullptr;       // totals partials, then the metric's scratch
    uint64_t* records = nullptr;   // one record block for the call's pass shape, or NULL: the workspace regions
    size_t record_words = 0;
    char* single = nullptr;        // b = 1 group buffer (NULL: single columns take the adding passes)
    int32_t single_group = 0;
};

dm_status query_args(const dm_handle* h, const void* Z, int32_t z_dtype, int32_t b, const void* Out, int* zkind) {
    if (!h || !Z || !Out || b < 1 || b > MAX_B) return DM_ERR_ARG;
    if (h->multi) return DM_ERR_STATE;
    {
        const dm_status zs = zkind_of(h, z_dtype, zkind);
        if (zs != DM_OK) return zs;
    }
    const size_t zbytes = (size_t)h->n * b * dtype_size(z_dtype);
    const size_t obytes = (size_t)h->n * b * (h->is_int ? 8 : 4);
    const char* zp = (const char*)Z;
    const char* op = (const char*)Out;
    if (zp < op + obytes && op < zp + zbytes) return DM_ERR_ARG;   // overlap
    return DM_OK;
}

// the record block of the call's pass shape
dm_status records_for(dm_handle* h, const QueryMem& q, const L1Shape& sh, uint64_t** out) {
    if (!q.records) return region_for(h, sh, out);
    if (sh.record_words > q.record_words) return DM_ERR_ARG;
    *out = q.records;
    return DM_OK;
}

dm_status matvec_impl(dm_handle* h, const void* Z, int zkind, int32_t b, void* Out, hipStream_t s,
                      const QueryMem& q) {
    char* sc = q.scratch;
    TotalsOut tot;
    tot.T0 = h->ctl->T0;
    tot.U = h->ctl->U;
    tot.zl1 = h->ctl->zl1;
    tot.status = &h->ctl->status;
    tot.partials = sc;
    char* rest = sc + al(totals_scratch_bytes(h->n, b));
    h->last = s;
    if (lp_metric(h->metric)) {
        // odd p: totals T0 and U (weights sum_k x^p), the moments T_1 .. T_(p-1)
        // of every coordinate, then one pass per coordinate
        const int pw = metric_power(h->metric);
        {
            ProfScope ps(h, DM_K_TOTALS, s);
            DM_TRY(launch_totals(h->is_int, zkind, Z, h->n, b, h->ws + h->L.rowsum, h->guard_scale, tot, s));
        }
        void* M = nullptr;
        DM_TRY(launch_lp_moments(h->is_int, zkind, pw, h->ws + h->L.xcopy, Z, h->n, h->d, b, rest, &M, s));
        LpPassArgs a;
        a.n = h->n;
        a.Z = Z;
        a.Out = Out;
        a.T0 = tot.T0;
        a.U = tot.U;
        a.mstride = (int64_t)h->d * b;
        a.chain = &h->ctl->chain;
        a.status = &h->ctl->status;
        {
            const L1Shape sh = lp_shape(h, b, zkind);
            dm_status rs = records_for(h, q, sh, &a.records);
            if (rs != DM_OK) return rs;
            a.record_words = sh.record_words;
            a.cls = sh.cls;
        }
        for (int32_t k = 0; k < h->d; ++k) {
            a.perm = h->at<uint32_t>(h->L.perm) + (size_t)k * h->L.ld;
            a.xs = h->ws + h->L.xs + (size_t)k * h->L.ld * 4;
            a.Mk = (const char*)M + (size_t)k * b * 8;
            a.first = k == 0;
            ProfScope ps(h, DM_K_L1_PASS, s);
            DM_TRY(launch_lp_pass(h->is_int, zkind, pw, b, a, s));
        }
    } else if (sf_metric(h->metric)) {
        // the single-moment forms on matrix cores sum z and w z inside their
        // moments kernel; the others take the totals kernel first
        const int form = sf_form(h->metric);
        const bool fuse = sf_fuses_totals(form, h->is_int, h->d, b, Z);
        if (!fuse) {
            ProfScope ps(h, DM_K_TOTALS, s);
            DM_TRY(launch_totals(h->is_int, zkind, Z, h->n, b, h->ws + h->L.rowsum, h->guard_scale, tot, s));
        }
        SfQuery q;
        q.X = h->ws + h->L.xcopy;
        q.LX = (h->metric == DM_KL || h->metric == DM_CE) ? h->at<double>(h->L.logx) : nullptr;
        q.centre = h->ws + h->L.centre;
        q.Z = Z;
        q.n = h->n;
        q.d = h->d;
        q.b = b;
        q.T0 = tot.T0;
        q.U = nullptr;
        q.a = nullptr;
        q.W = nullptr;
        q.alpha = 1.0;
        q.Out = Out;
        const double* weights = h->at<double>(h->L.rowsum);
        const double* W = h->at<double>(h->L.mat + (size_t)h->d * h->d * 8);
        switch (h->metric) {
        case DM_KL:   // -H_i sum z - sum_k x_ik S_k (Algorithm 4)
            q.alpha = -1.0;
            q.a = weights;
            break;
        case DM_CE:   // -sum_k x_ik S_k
            q.alpha = -1.0;
            break;
        case DM_MAHA2:   // q_i sum z + sum_j q_j z_j - x~_i^T (M + M^T) sum_j z_j x~_j
            q.W = W;
            q.a = weights;
            q.U = (const double*)tot.U;
            if (fuse) q.wu = weights;
            break;
        case DM_BILINEAR:   // x_i^T M sum_j z_j x_j (Algorithms 8 and 9)
            q.W = W;
            q.centre = nullptr;
            break;
        default:
            break;
        }
        if (fuse) q.status = &h->ctl->status;
        ProfScope ps(h, DM_K_SORTFREE, s);
        DM_TRY(launch_sf_query(form, metric_power(h->metric), h->is_int, zkind, q, rest, s));
    } else if (l1_pass_metric(h->metric)) {
        {
            ProfScope ps(h, DM_K_TOTALS, s);
            DM_TRY(launch_totals(h->is_int, zkind, Z, h->n, b, h->ws + h->L.rowsum, h->guard_scale, tot, s));
        }
        L1PassArgs a;
        a.n = h->n;
        a.Z = Z;
        a.Out = Out;
        a.T0 = tot.T0;
        a.U = tot.U;
        a.chain = &h->ctl->chain;
        a.status = &h->ctl->status;
        {
            const int v = variant_for(h, kind_index(h->is_int, zkind), log2_pad(b));
            const L1Shape sh = l1_shape(h->n, b, h->is_int, zkind, v);
            dm_status rs = records_for(h, q, sh, &a.records);
            if (rs != DM_OK) return rs;
            a.record_words = sh.record_words;
            a.cls = sh.cls;
            a.variant = v;
        }
        const size_t vsz = 4;
        // one column: each pass writes its values in point order to a buffer
        // of its own (the workspace's group buffer), and after each group of G
        // coordinates one coalesced sweep adds the group's buffers into Out
        const bool single = b == 1 && q.single;
        const int32_t G = single ? q.single_group : 1;
        char* single_buf = q.single;
        const size_t osz = h->is_int ? 8 : 4;
        if (single) {
            const L1Shape sh = l1_single_shape(h->n, h->is_int, zkind, a.variant);
            dm_status rs = records_for(h, q, sh, &a.records);
            if (rs != DM_OK) return rs;
            a.record_words = sh.record_words;
            a.cls = sh.cls;
            a.out_mode = OUT_FRESH;
        }
        for (int32_t k = 0; k < h->d; ++k) {
            a.perm = h->at<uint32_t>(h->L.perm) + (size_t)k * h->L.ld;
            a.xs = h->ws + h->L.xs + (size_t)k * h->L.ld * vsz;
            a.first = k == 0;
            if (single) a.Out = single_buf + (size_t)(k % G) * h->L.ld * osz;
            {
                ProfScope ps(h, DM_K_L1_PASS, s);
                DM_TRY(launch_l1_pass(h->is_int, zkind, b, a, s));
            }
            if (single && (k % G == G - 1 || k == h->d - 1)) {
                const int32_t k0 = k - k % G;
                DM_TRY(launch_l1_combine(h->is_int, h->L.ld, single_buf, h->n, k - k0 + 1, k0 == 0, tot.U, Out, s));
            }
        }
        // TV(x, y) = l1(x, y) / 2 (the TV theorem of Appendix A.3); the
        // halving is exact in floating point
        if (h->metric == DM_TV) DM_TRY(launch_scale_f32((float*)Out, (size_t)h->n * b, 0.5f, s));
    } else {
        ProfScope ps(h, DM_K_L2, s);
        DM_TRY(launch_l2sq(h->is_int, zkind, h->ws + h->L.xcopy, h->ws + h->L.rownrm, h->n, h->d, Z, b, Out, rest,
                           tot, h->guard_scale, s));
    }
    return DM_OK;
}

}  // namespace

extern "C" {

dm_status dm_matvec(dm_handle* h, const void* Z, int32_t z_dtype, int32_t b, void* Out, void* stream) {
    int zkind = 0;
    dm_status st = query_args(h, Z, z_dtype, b, Out, &zkind);
    if (st != DM_OK) return st;
    QueryMem q;
    q.scratch = h->ws + h->L.qscratch;
    if (h->L.single_bytes) {
        q.single = h->ws + h->L.single;
        q.single_group = h->L.single_group;
    }
    hipStream_t s = (hipStream_t)stream;
    // profiling brackets every launch with events: run those queries eagerly
    if (!h->use_graphs || h->prof) return matvec_impl(h, Z, zkind, b, Out, s, q);
    for (auto& g : h->graphs)
        if (g.Z == Z && g.Out == Out && g.b == b && g.zkind == zkind) {
            g.used = ++h->graph_clock;
            DM_TRY(hipGraphLaunch(g.exec, s));
            h->last = s;
            return DM_OK;
        }
    // record the query's launches (nothing runs during the capture), then
    // launch the graph on the caller's stream
    if (!h->cap) DM_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    DM_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    st = matvec_impl(h, Z, zkind, b, Out, h->cap, q);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap, &graph);
    if (st != DM_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != DM_OK ? st : from_hip(ec);
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return from_hip(ei);
    if ((int)h->graphs.size() == dm_handle::GRAPHS) {
        auto lru = std::min_element(h->graphs.begin(), h->graphs.end(),
                                    [](const dm_handle::Graph& a, const dm_handle::Graph& c) { return a.used < c.used; });
        // a replay of the evicted graph may still be queued on some stream:
        // wait for the handle's last stream before destroying it
        if (h->last) DM_TRY(hipStreamSynchronize(h->last));
        (void)hipGraphExecDestroy(lru->exec);
        h->graphs.erase(lru);
    }
    h->graphs.push_back(dm_handle::Graph{Z, Out, b, zkind, exec, ++h->graph_clock});
    DM_TRY(hipGraphLaunch(exec, s));
    h->last = s;
    return DM_OK;
}

dm_status dm_matvec_static(dm_handle* h, const void* Z, int32_t z_dtype, int32_t b, void* Out, void* stream) {
    int zkind = 0;
    dm_status st = query_args(h, Z, z_dtype, b, Out, &zkind);
    if (st != DM_OK) return st;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DM_ERR_DEVICE;
    if (dev != h->device) return DM_ERR_ARG;   // the array of the handle's device must be current
    // plan the call's memory inside the static array: query scratch, the
    // record block of the pass shape, and (b = 1, l1 / TV) as many
    // coordinates of the group buffer as fit
    QueryMem q;
    size_t at = al(query_scratch_bytes(h->n, h->d, h->metric, b));
    size_t words = 0;
    if (l1_pass_metric(h->metric)) {
        const int v = variant_for(h, kind_index(h->is_int, zkind), log2_pad(b));
        words = l1_shape(h->n, b, h->is_int, zkind, v).record_words;
        if (b == 1) words = std::max(words, l1_single_shape(h->n, h->is_int, zkind, v).record_words);
    } else if (lp_metric(h->metric)) {
        words = lp_shape(h, b, zkind).record_words;
    }
    const size_t rec_at = at;
    at += al(words * 8);
    if (at > STATIC_SCRATCH_BYTES) return DM_ERR_ARG;   // beyond the array: use dm_matvec
    char* base = nullptr;
    if (static_scratch(&base) != hipSuccess) return DM_ERR_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    q.scratch = base;
    if (words) {
        q.records = (uint64_t*)(base + rec_at);
        q.record_words = words;
        // the array keeps the last call's records (any handle's): start from
        // zero words, which carry no pass tag
        DM_TRY(launch_fill_u32((uint32_t*)q.records, 0u, words * 2, s));
    }
    if (b == 1 && l1_pass_metric(h->metric)) {
        const size_t per = (size_t)h->L.ld * (h->is_int ? 8 : 4);
        const size_t g = (STATIC_SCRATCH_BYTES - at) / per;
        if (g >= 1) {
            q.single = base + at;
            q.single_group = (int32_t)std::min<size_t>(g, (size_t)h->d);
        }
    }
    return matvec_impl(h, Z, zkind, b, Out, s, q);
}

dm_status dm_set_variant(dm_handle* h, int32_t b, int32_t z_dtype, int32_t variant) {
    if (!h || b < 1 || b > MAX_B || variant < 0 || variant >= L1_VARIANTS) return DM_ERR_ARG;
    if (h->multi) return DM_ERR_STATE;
    if (!l1_pass_metric(h->metric)) return DM_ERR_ARG;
    int zkind = 0;
    const dm_status st = zkind_of(h, z_dtype, &zkind);
    if (st != DM_OK) return st;
    h->variant[kind_index(h->is_int, zkind)][log2_pad(b)] = (int8_t)variant;
    drop_graphs(h);   // captured queries hold the old variant's launches
    return DM_OK;
}

dm_status dm_get_variant(dm_handle* h, int32_t b, int32_t z_dtype, int32_t* variant) {
    if (!h || !variant || b < 1 || b > MAX_B) return DM_ERR_ARG;
    if (h->multi) return DM_ERR_STATE;
    if (!l1_pass_metric(h->metric)) return DM_ERR_ARG;
    int zkind = 0;
    const dm_status st = zkind_of(h, z_dtype, &zkind);
    if (st != DM_OK) return st;
    *variant = variant_for(h, kind_index(h->is_int, zkind), log2_pad(b));
    return DM_OK;
}

int32_t dm_variant_count(void) { return L1_VARIANTS; }

dm_status dm_tune(dm_handle* h, int32_t b, int32_t z_dtype, int32_t reps, void* stream, int32_t* chosen,
                  double* ms_per_pass) {
    if (!h || b < 1 || b > MAX_B || reps < 1 || reps > 4096) return DM_ERR_ARG;
    if (h->multi) return DM_ERR_STATE;
    if (!l1_pass_metric(h->metric)) return DM_ERR_ARG;
    int zkind = 0;
    dm_status st = zkind_of(h, z_dtype, &zkind);
    if (st != DM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int kind = kind_index(h->is_int, zkind), lg = log2_pad(b);
    const size_t zb = (size_t)h->n * b * dtype_size(z_dtype);
    const size_t ob = (size_t)h->n * b * (h->is_int ? 8 : 4);
    void* Zt = nullptr;
    void* Ot = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 1e300;
    int bestv = 0;
    // time every variant on this handle's own sorted coordinates with a zero
    // right-hand side (the pass time does not depend on the values)
    auto run = [&]() -> dm_status {
        if (hipMalloc(&Zt, zb) != hipSuccess || hipMalloc(&Ot, ob) != hipSuccess) return DM_ERR_NOMEM;
        DM_TRY(launch_fill_u32((uint32_t*)Zt, 0u, zb / 4, s));
        DM_TRY(launch_fill_u32((uint32_t*)Ot, 0u, ob / 4, s));
        DM_TRY(hipEventCreate(&e0));
        DM_TRY(hipEventCreate(&e1));
        L1PassArgs a;
        a.n = h->n;
        a.Z = Zt;
        a.Out = Ot;
        a.T0 = h->ctl->T0;
        a.U = h->ctl->U;
        a.chain = &h->ctl->chain;
        a.status = &h->ctl->status;
        a.first = 0;
        // a single column runs the OUT_FRESH passes
        a.out_mode = b == 1 ? OUT_FRESH : OUT_ADD;
        for (int v = 0; v < L1_VARIANTS; ++v) {
            const L1Shape sh =
                b == 1 ? l1_single_shape(h->n, h->is_int, zkind, v) : l1_shape(h->n, b, h->is_int, zkind, v);
            const dm_status rs = region_for(h, sh, &a.records);
            if (rs != DM_OK) return rs;
            a.record_words = sh.record_words;
            a.cls = sh.cls;
            a.variant = v;
            for (int i = -1; i < reps; ++i) {   // one untimed pass, then reps timed ones
                if (i == 0) DM_TRY(hipEventRecord(e0, s));
                const int32_t k = (i + 1) % h->d;
                a.perm = h->at<uint32_t>(h->L.perm) + (size_t)k * h->L.ld;
                a.xs = h->ws + h->L.xs + (size_t)k * h->L.ld * 4;
                DM_TRY(launch_l1_pass(h->is_int, zkind, b, a, s));
            }
            DM_TRY(hipEventRecord(e1, s));
            DM_TRY(hipEventSynchronize(e1));
            float t = 0.0f;
            DM_TRY(hipEventElapsedTime(&t, e0, e1));
            const double per = (double)t / reps;
            if (ms_per_pass) ms_per_pass[v] = per;
            if (per < best) {
                best = per;
                bestv = v;
            }
        }
        return DM_OK;
    };
    st = run();
    if (hipStreamSynchronize(s) != hipSuccess && st == DM_OK) st = DM_ERR_DEVICE;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (Zt) (void)hipFree(Zt);
    if (Ot) (void)hipFree(Ot);
    if (st != DM_OK) return st;
    h->variant[kind][lg] = (int8_t)bestv;
    drop_graphs(h);
    cache_store(h, kind, lg, bestv);
    if (chosen) *chosen = bestv;
    h->last = s;
    return DM_OK;
}

dm_status dm_lowrank(dm_handle* h, int32_t rank, int32_t block, int32_t iters, const double* Omega, double* U,
                     double* lam, void* stream, int32_t* sweeps) {
    if (!h || !Omega || !U || !lam) return DM_ERR_ARG;
    if (h->multi) return DM_ERR_STATE;
    if (h->is_int) return DM_ERR_DTYPE;
    if (!h->symmetric) return DM_ERR_STATE;   // the Rayleigh-Ritz step needs A = A^T
    if (block < 1 || block > lr_max_block() || iters < 1 || rank < 1 || rank > lr_max_block()) return DM_ERR_ARG;
    const int64_t K64 = (int64_t)block * iters;
    if (K64 > lr_max_basis() || rank > K64) return DM_ERR_ARG;
    const int K = (int)K64, B = block;
    const int64_t n = h->n;
    hipStream_t s = (hipStream_t)stream;

    // one allocation for the basis (iters blocks, plus one for the last
    // product), the FP32 staging of the products, and the small matrices
    const size_t nb = (size_t)n * B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_basis = take(nb * (iters + 1) * sizeof(double));
    const size_t o_zf = take(nb * sizeof(float));
    const size_t o_yf = take(nb * sizeof(float));
    const size_t o_part = take(lr_gram_scratch_doubles(n, B, B, iters) * sizeof(double));
    const size_t o_T = take((size_t)K * K * sizeof(double));
    const size_t o_V = take((size_t)K * K * sizeof(double));
    const size_t o_T2 = take((size_t)K * K * sizeof(double));
    const size_t o_w = take((size_t)K * sizeof(double));
    const size_t o_G = take((size_t)B * B * sizeof(double));
    const size_t o_X = take((size_t)B * B * sizeof(double));
    const size_t o_C = take((size_t)K * B * sizeof(double));
    const size_t o_Vk = take((size_t)K * rank * sizeof(double));
    const size_t o_sw = take(sizeof(int));
    char* mem = nullptr;
    if (hipMalloc(&mem, off) != hipSuccess) return DM_ERR_NOMEM;
    double* basis = (double*)(mem + o_basis);
    float* Zf = (float*)(mem + o_zf);
    float* Yf = (float*)(mem + o_yf);
    double* part = (double*)(mem + o_part);
    double* T = (double*)(mem + o_T);
    double* V = (double*)(mem + o_V);
    double* T2 = (double*)(mem + o_T2);
    double* w = (double*)(mem + o_w);
    double* G = (double*)(mem + o_G);
    double* X = (double*)(mem + o_X);
    double* C = (double*)(mem + o_C);
    double* Vk = (double*)(mem + o_Vk);
    int* d_sweeps = (int*)(mem + o_sw);
    auto Qb = [&](int i) { return basis + (size_t)i * nb; };
    uint32_t* status = &h->ctl->status;
    // a column is dropped when it is in the span of the earlier ones to
    // relative accuracy 1e-10
    const double rel = 1e-20;

    // The products run on the FP32 copy split into a block of 32k columns and
    // the rest (B = 40: 32 + 8), queried one after the other: a 128-byte row
    // fills one cache line and a 32-byte row sits inside one, where every
    // 160-byte row of the 40-column block spans two 128-byte lines.
    const int B1 = B > 32 && B % 32 != 0 ? B / 32 * 32 : B;
    int sw_used = 0;
    auto run = [&]() -> dm_status {
        const double* Qprev = Omega;
        for (int j = 0; j <= iters; ++j) {
            // Y = A Q_{j-1} (A Omega for j = 0), through the FP32 query
            double* Y = Qb(j);
            DM_TRY(lr_cvt(Qprev, Zf, n, B, B1, s));
            dm_status ms = dm_matvec(h, Zf, DM_F32, B1, Yf, s);
            if (ms == DM_OK && B1 < B) ms = dm_matvec(h, Zf + (size_t)n * B1, DM_F32, B - B1, Yf + (size_t)n * B1, s);
            if (ms != DM_OK) return ms;
            DM_TRY(lr_cvt(Yf, Y, n, B, B1, s));
            // Block classical Gram-Schmidt against Q_0 .. Q_{j-1}, twice: every
            // coefficient block Q_i^T Y first, then one update
            // Y -= sum_i Q_i C_i that moves Y once.  The first pass's
            // coefficients Q_i^T (A Q_{j-1}) are exactly the Rayleigh-Ritz
            // blocks T[i][j-1], so they are written straight into T (rows
            // i B .. of column block j - 1, leading dimension K).
            if (j > 0) DM_TRY(lr_gram_blocks(Qb(0), nb, j, B, Y, B, n, part, T + (size_t)(j - 1) * B, K, 1.0, s));
            if (j == iters) break;
            if (j > 0) {
                DM_TRY(lr_update_blocks(Y, B, Qb(0), nb, j, B, T + (size_t)(j - 1) * B, K, -1.0, 1.0, n, s));
                DM_TRY(lr_gram_blocks(Qb(0), nb, j, B, Y, B, n, part, C, B, 1.0, s));
                DM_TRY(lr_update_blocks(Y, B, Qb(0), nb, j, B, C, B, -1.0, 1.0, n, s));
            }
            // Cholesky QR, twice
            for (int pass = 0; pass < 2; ++pass) {
                DM_TRY(lr_gram_blocks(Y, 0, 1, B, Y, B, n, part, G, B, 1.0, s));
                DM_TRY(lr_cholinv(G, B, rel, X, status, s));
                DM_TRY(lr_update_rows(Y, B, Y, B, X, B, 1.0, 0.0, n, s));
            }
            Qprev = Y;
        }
        DM_TRY(lr_symm(T, K, B, s));
        int sw_host = 0;
        DM_TRY(lr_eig(T, T2, V, w, K, 60, 1e-14, d_sweeps, &sw_host, s));
        sw_used = sw_host;
        DM_TRY(lr_topk(w, V, K, rank, lam, Vk, s));
        // U = Q Vk = sum_i Q_i Vk_i in one pass over U
        DM_TRY(lr_update_blocks(U, rank, Qb(0), nb, iters, B, Vk, rank, 1.0, 0.0, n, s));
        return DM_OK;
    };
    dm_status st = run();
    if (hipStreamSynchronize(s) != hipSuccess && st == DM_OK) st = DM_ERR_DEVICE;
    (void)hipFree(mem);
    if (sweeps) *sweeps = sw_used;
    h->last = s;
    if (st != DM_OK) return st;
    return dm_sync(h);
}

dm_status dm_embed_l2(const void* X, int64_t n, int32_t d, int32_t dtype, const double* G, int32_t k, float* Xout,
                      void* stream) {
    if (!X || !G || !Xout || n < 1 || d < 1 || k < 1 || k > 65536 || !valid_dtype(dtype)) return DM_ERR_ARG;
    const char* xp = (const char*)X;
    const char* op = (const char*)Xout;
    const size_t xb = (size_t)n * d * dtype_size(dtype), ob = (size_t)n * k * sizeof(float);
    if (xp < op + ob && op < xp + xb) return DM_ERR_ARG;   // overlap
    int dev = 0;
    const dm_status st = device_ready(&dev);
    if (st != DM_OK) return st;
    DM_TRY(launch_embed_l2(dtype, X, n, d, G, k, Xout, (hipStream_t)stream));
    return DM_OK;
}

dm_status dm_sync(dm_handle* h) {
    if (!h) return DM_ERR_ARG;
    if (hipStreamSynchronize(h->last) != hipSuccess) return DM_ERR_DEVICE;
    uint32_t st = 0;
    if (hipMemcpy(&st, &h->ctl->status, 4, hipMemcpyDeviceToHost) != hipSuccess) return DM_ERR_DEVICE;
    if (st) {
        const uint32_t zero = 0;
        if (hipMemcpy(&h->ctl->status, &zero, 4, hipMemcpyHostToDevice) != hipSuccess) return DM_ERR_DEVICE;
    }
    if (st & QF_NONFINITE) return DM_ERR_NONFINITE;
    if (st & QF_OVERFLOW) return DM_ERR_OVERFLOW;
    if (st & QF_STALL) return DM_ERR_DEVICE;
    return DM_OK;
}

dm_status dm_info(const dm_handle* h, int64_t* n, int32_t* d, int32_t* metric, int32_t* dtype) {
    if (!h) return DM_ERR_ARG;
    if (n) *n = h->n;
    if (d) *d = h->d;
    if (metric) *metric = h->metric;
    if (dtype) *dtype = h->dtype;
    return DM_OK;
}

dm_status dm_copy_sorted(const dm_handle* h, uint32_t* perm, uint32_t* rank, void* xs, void* stream) {
    if (!h) return DM_ERR_ARG;
    if (h->multi) return DM_ERR_STATE;
    if (!sorted_metric(h->metric)) return DM_ERR_STATE;
    hipStream_t s = (hipStream_t)stream;
    const size_t w = (size_t)h->n * 4, sp = (size_t)h->L.ld * 4;
    if (perm) DM_TRY(hipMemcpy2DAsync(perm, w, h->ws + h->L.perm, sp, w, h->d, hipMemcpyDeviceToDevice, s));
    // the inverse permutations are formed on request (no query reads them)
    if (rank) DM_TRY(launch_rank_invert(h->at<uint32_t>(h->L.perm), h->L.ld, h->n, h->d, rank, h->n, s));
    if (xs) {
        DM_TRY(hipMemcpy2DAsync(xs, w, h->ws + h->L.xs, sp, w, h->d, hipMemcpyDeviceToDevice, s));
        // float values are kept relative to their coordinate's centre
        if (!h->is_int) DM_TRY(launch_add_centre((float*)xs, h->n, h->d, h->n, h->at<float>(h->L.c32), s));
    }
    return DM_OK;
}

dm_status dm_profile_enable(dm_handle* h, int32_t on) {
    if (!h) return DM_ERR_ARG;
    h->prof = on != 0;
    h->ev_used = 0;
    for (int c = 0; c < DM_K_CLASSES; ++c) {
        h->prof_ms[c] = 0.0;
        h->prof_n[c] = 0;
    }
    return DM_OK;
}

dm_status dm_profile_read(dm_handle* h, int32_t kernel_class, double* total_ms, int64_t* launches) {
    if (!h || kernel_class < 0 || kernel_class >= DM_K_CLASSES) return DM_ERR_ARG;
    for (size_t i = 0; i < h->ev_used; ++i) {
        auto& e = h->evs[i];
        float ms = 0.0f;
        if (hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess)
            return DM_ERR_DEVICE;
        h->prof_ms[e.cls] += ms;
        h->prof_n[e.cls] += 1;
    }
    h->ev_used = 0;
    if (total_ms) *total_ms = h->prof_ms[kernel_class];
    if (launches) *launches = h->prof_n[kernel_class];
    return DM_OK;
}

dm_status dm_copy_probe(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || bytes == 0 || bytes % 16 != 0) return DM_ERR_ARG;
    if (((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return DM_ERR_ARG;
    const char* d = (const char*)dst;
    const char* s = (const char*)src;
    if (d < s + bytes && s < d + bytes) return DM_ERR_ARG;
    DM_TRY(launch_copy_probe(dst, src, bytes, (hipStream_t)stream));
    return DM_OK;
}

dm_status dm_gather_probe(const uint32_t* perm, const float* Z, float* Out, int64_t n, int32_t b, void* stream) {
    if (!perm || !Z || !Out || n < 1 || n > (int64_t)UINT32_MAX) return DM_ERR_ARG;
    if (b < 4 || b > 64 || (b & (b - 1)) != 0) return DM_ERR_ARG;
    if (((uintptr_t)Z | (uintptr_t)Out) % 16 != 0 || (uintptr_t)perm % 4 != 0) return DM_ERR_ARG;
    const char* z = (const char*)Z;
    const char* o = (const char*)Out;
    const size_t bytes = (size_t)n * b * 4;
    if (o < z + bytes && z < o + bytes) return DM_ERR_ARG;
    DM_TRY(launch_gather_probe(perm, Z, Out, n, b, (hipStream_t)stream));
    return DM_OK;
}

void dm_free(dm_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->last);
    release(h);
}

}  // extern "C"

// ===========================================================================
// many datasets in one query
// ===========================================================================
namespace {

struct MultiSet {
    int64_t n = 0, ld = 0, base = 0;   // base: first key of the dataset in the concatenated arrays
    int32_t d = 0, dtype = 0;
    int32_t seg0 = 0;                  // its first segment (coordinate 0) of the segmented sort
    bool is_int = false;
    size_t rowsum = 0, rownrm = 0, kmin = 0, kmax = 0;
    double guard = 0.0;
};

struct MultiPlan {
    int32_t b = 0;
    bool vec = false;              // 16-byte row accesses (captured into the graph)
    int32_t rounds = 0;
    std::vector<int64_t> ntiles;   // [round][kind]
    std::vector<int> grids;
    std::vector<MultiTile*> tiles;
    std::vector<uint64_t*> records;
    uint64_t* tickets = nullptr;   // one per (round, kind)
    double* partials = nullptr;
    double* tot = nullptr;         // per dataset: T0 (b) and U (b)
    int variant = 0;               // tile variant of the plan's pass launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct MultiLayout {
    size_t perm = 0, xs = 0, ids = 0, k1 = 0, v1 = 0, counts = 0, flags = 0;
    size_t key_off = 0, key_len = 0, tile_off = 0, tile_seg = 0, seg_int = 0;
    size_t centre = 0;             // per segment: FP32 centre of a float coordinate
    // what queries use: control block, descriptors, totals block table, and
    // the plan area (sized for the largest b), all in the workspace
    size_t ctl = 0, ds = 0, blk = 0;
    size_t tickets = 0, tot = 0, partials = 0;
    size_t plan = 0, plan_bytes = 0;
    int nblk = 0;
    int64_t total_keys = 0;
    uint32_t ntiles = 0;
    int32_t nseg = 0;
    size_t total = 0;
};

}  // namespace

struct MultiState {
    std::vector<MultiSet> sets;
    MultiLayout L;
    int32_t maxd = 0;
    MultiDs* d_ds = nullptr;     // device descriptors
    MultiDs* h_ds = nullptr;     // pinned host mirror (source of the captured upload)
    uint32_t* d_blk = nullptr;   // dataset of every totals block
    int nblk = 0;
    MultiPlan plan;
    int8_t variant[7] = {0, 0, 0, 0, 0, 0, 0};   // tile variant per log2 of the padded b (set or tuned)
    hipStream_t cap = nullptr;   // capture stream
    hipEvent_t done = nullptr;   // recorded after every graph launch
    bool launched = false;
};

namespace {

void free_plan(MultiPlan& p) {
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    p = MultiPlan();
}

dm_status check_multi(const dm_dataset* sets, int32_t count, std::vector<MultiSet>* out, MultiLayout* L) {
    if (!sets || count < 1) return DM_ERR_ARG;
    std::vector<MultiSet> v((size_t)count);
    int64_t keys = 0;
    for (int32_t i = 0; i < count; ++i) {
        const dm_dataset& ds = sets[i];
        if (ds.n < 1 || ds.d < 1 || ds.metric != DM_L1 || !valid_dtype(ds.dtype)) return DM_ERR_ARG;
        v[i].n = ds.n;
        v[i].d = ds.d;
        v[i].dtype = ds.dtype;
        v[i].is_int = int_dtype(ds.dtype);
        v[i].ld = (ds.n + 63) / 64 * 64;
        v[i].base = keys;
        keys += (int64_t)ds.d * v[i].ld;
        if (keys >= (int64_t)1 << 32) return DM_ERR_ARG;   // 32-bit sort positions
    }
    MultiLayout M;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += al(bytes);
        return at;
    };
    M.total_keys = keys;
    const size_t arr = (size_t)keys * 4;
    M.perm = take(arr);
    M.xs = take(arr);
    M.ids = take(arr);
    int32_t nseg = 0;
    uint32_t ntiles = 0;
    for (auto& m : v) {
        m.rowsum = take((size_t)m.n * 8);
        m.rownrm = take((size_t)m.n * 8);
        m.kmin = take((size_t)m.d * 4);
        m.kmax = take((size_t)m.d * 4);
        m.seg0 = nseg;
        nseg += m.d;
        ntiles += (uint32_t)m.d * (uint32_t)((m.n + SORT_TILE - 1) / SORT_TILE);
    }
    M.nseg = nseg;
    M.ntiles = ntiles;
    M.flags = take(16);
    M.key_off = take((size_t)nseg * 8);
    M.key_len = take((size_t)nseg * 8);
    M.tile_off = take((size_t)(nseg + 1) * 4);
    M.tile_seg = take((size_t)ntiles * 4);
    M.seg_int = take((size_t)nseg);
    M.centre = take((size_t)nseg * 4);
    M.k1 = take(arr);
    M.v1 = take(arr);
    M.counts = take((size_t)ntiles * 256 * 4);
    int maxd = 0;
    for (auto& m : v) {
        M.nblk += (int)((m.n + multi_totals_rows() - 1) / multi_totals_rows());
        maxd = std::max(maxd, m.d);
    }
    M.ctl = take(sizeof(Ctl));
    M.ds = take((size_t)count * sizeof(MultiDs));
    M.blk = take((size_t)M.nblk * 4);
    M.tickets = take((size_t)maxd * 2 * 8);
    M.tot = take((size_t)count * 2 * MAX_B * 8);
    M.partials = take((size_t)M.nblk * MAX_B * 3 * 8 + 8);
    // per (round, kind): the tile table and the record region of that
    // round's launch; both depend on b and the tile variant through the tile size
    for (int32_t b = 1; b <= MAX_B; ++b)
        for (int var = 0; var < MULTI_VARIANTS; ++var) {
        size_t bytes = 0;
        for (int k = 0; k < maxd; ++k)
            for (int kind = 0; kind < 2; ++kind) {
                const int tr = multi_tile_ranks(b, kind == 1, var);
                int64_t nt = 0;
                for (auto& m : v)
                    if (m.is_int == (kind == 1) && m.d > k) nt += (m.n + tr - 1) / tr;
                if (nt == 0) continue;
                bytes += al((size_t)nt * sizeof(MultiTile)) + al(multi_record_words(nt, b, kind == 1) * 8);
            }
        M.plan_bytes = std::max(M.plan_bytes, bytes);
        }
    M.plan = take(M.plan_bytes);
    M.total = o;
    if (out) *out = std::move(v);
    if (L) *L = M;
    return DM_OK;
}

// Build the round tables, record regions and the captured graph for b and
// tile variant v.
dm_status build_plan(dm_handle* h, int32_t b, bool vec, int v) {
    MultiState* m = h->multi;
    MultiPlan& p = m->plan;
    if (m->launched) DM_TRY(hipEventSynchronize(m->done));
    free_plan(p);
    p.b = b;
    p.vec = vec;
    p.variant = v;
    p.rounds = m->maxd;
    const int nsets = (int)m->sets.size();
    // per-dataset totals storage and descriptors
    {
        p.tot = h->at<double>(m->L.tot);
        p.partials = h->at<double>(m->L.partials);
        p.tickets = h->at<uint64_t>(m->L.tickets);
        DM_TRY(launch_fill_u32((uint32_t*)p.tickets, 0u, (size_t)p.rounds * 4, m->cap));
    }
    size_t at = m->L.plan;   // tile tables and record regions, carved in order
    for (int s = 0; s < nsets; ++s) {
        m->h_ds[s].T0 = p.tot + (size_t)s * 2 * b;
        m->h_ds[s].U = p.tot + (size_t)s * 2 * b + b;
    }
    // datasets largest first inside every round, so long segments start early
    std::vector<int> order(nsets);
    for (int s = 0; s < nsets; ++s) order[s] = s;
    std::sort(order.begin(), order.end(), [&](int a, int c) { return m->sets[a].n > m->sets[c].n; });
    p.ntiles.assign((size_t)p.rounds * 2, 0);
    p.grids.assign((size_t)p.rounds * 2, 0);
    p.tiles.assign((size_t)p.rounds * 2, nullptr);
    p.records.assign((size_t)p.rounds * 2, nullptr);
    for (int k = 0; k < p.rounds; ++k)
        for (int kind = 0; kind < 2; ++kind) {
            const int tr = multi_tile_ranks(b, kind == 1, v);
            std::vector<MultiTile> t;
            for (int s : order) {
                const MultiSet& ms = m->sets[s];
                if (ms.is_int != (kind == 1) || ms.d <= k) continue;
                const int64_t nt = (ms.n + tr - 1) / tr;
                for (int64_t i = 0; i < nt; ++i) t.push_back(MultiTile{(uint32_t)s, (uint32_t)i});
            }
            const size_t ix = (size_t)k * 2 + kind;
            p.ntiles[ix] = (int64_t)t.size();
            if (t.empty()) continue;
            const size_t words = multi_record_words((int64_t)t.size(), b, kind == 1);
            if (at + al(t.size() * sizeof(MultiTile)) + al(words * 8) > m->L.plan + m->L.plan_bytes)
                return DM_ERR_STATE;   // cannot happen: the plan area is sized for every b
            void* q = h->ws + at;
            at += al(t.size() * sizeof(MultiTile));
            p.tiles[ix] = (MultiTile*)q;
            DM_TRY(hipMemcpyAsync(q, t.data(), t.size() * sizeof(MultiTile), hipMemcpyHostToDevice, m->cap));
            q = h->ws + at;
            at += al(words * 8);
            p.records[ix] = (uint64_t*)q;
            DM_TRY(launch_fill_u32((uint32_t*)q, 0u, words * 2, m->cap));
            p.grids[ix] = multi_grid((int64_t)t.size(), b, kind == 1, v);
            DM_TRY(hipStreamSynchronize(m->cap));   // the host vector dies with this scope
        }
    // capture: descriptor upload, totals, every round
    DM_TRY(hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipMemcpyAsync(m->d_ds, m->h_ds, (size_t)nsets * sizeof(MultiDs), hipMemcpyHostToDevice, m->cap);
    if (e == hipSuccess)
        e = launch_multi_totals(m->d_ds, m->d_blk, m->nblk, nsets, b, p.partials, &h->ctl->status, m->cap);
    for (int k = 0; k < p.rounds && e == hipSuccess; ++k)
        for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
            const size_t ix = (size_t)k * 2 + kind;
            if (p.ntiles[ix] == 0) continue;
            e = launch_multi_pass(kind == 1, b, m->d_ds, p.tiles[ix], p.ntiles[ix], k, p.tickets + ix, p.records[ix],
                                  p.grids[ix], p.vec, &h->ctl->status, v, m->cap);
        }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(m->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return from_hip(e != hipSuccess ? e : e2);
    }
    p.graph = g;
    DM_TRY(hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0));
    return DM_OK;
}

void release_multi(MultiState* m) {
    if (!m) return;
    if (m->launched) (void)hipEventSynchronize(m->done);
    free_plan(m->plan);
    if (m->h_ds) (void)hipHostFree(m->h_ds);
    if (m->done) (void)hipEventDestroy(m->done);
    if (m->cap) (void)hipStreamDestroy(m->cap);
    delete m;
}

}  // namespace

extern "C" {

dm_status dm_workspace_size_multi(const dm_dataset* sets, int32_t count, size_t* bytes) {
    if (!bytes) return DM_ERR_ARG;
    MultiLayout L;
    dm_status st = check_multi(sets, count, nullptr, &L);
    if (st != DM_OK) return st;
    *bytes = L.total;
    return DM_OK;
}

dm_status dm_prepare_multi(const dm_dataset* sets, int32_t count, void* workspace, size_t ws_bytes, void* stream,
                           dm_handle** out) {
    if (!out) return DM_ERR_ARG;
    *out = nullptr;
    std::vector<MultiSet> v;
    MultiLayout L;
    dm_status st = check_multi(sets, count, &v, &L);
    if (st != DM_OK) return st;
    for (int32_t i = 0; i < count; ++i)
        if (!sets[i].X) return DM_ERR_ARG;
    if (workspace && (ws_bytes < L.total || ((uintptr_t)workspace % ALIGN) != 0)) return DM_ERR_ARG;
    int dev = 0;
    if ((st = device_ready(&dev)) != DM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    dm_handle* h = new (std::nothrow) dm_handle();
    if (!h) return DM_ERR_NOMEM;
    MultiState* m = new (std::nothrow) MultiState();
    if (!m) {
        delete h;
        return DM_ERR_NOMEM;
    }
    h->multi = m;
    h->device = dev;
    h->metric = DM_L1;
    h->n = 0;
    for (auto& q : v) {
        h->n += q.n;
        m->maxd = std::max(m->maxd, q.d);
    }
    h->d = m->maxd;
    h->dtype = 0;
    m->sets = v;
    m->L = L;
    auto fail = [&](dm_status e) {
        release(h);
        return e;
    };
    if (workspace) {
        h->ws = (char*)workspace;
    } else {
        void* p = nullptr;
        if (hipMalloc(&p, L.total) != hipSuccess) return fail(DM_ERR_NOMEM);
        h->ws = (char*)p;
        h->owns_ws = true;
    }
    h->ctl = h->at<Ctl>(L.ctl);
    if (hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&m->done, hipEventDisableTiming) != hipSuccess)
        return fail(DM_ERR_DEVICE);
    Ctl init;
    std::memset(&init, 0, sizeof(init));
    if (hipMemcpyAsync(h->ctl, &init, sizeof(Ctl), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(DM_ERR_DEVICE);
    if (launch_fill_u32(h->at<uint32_t>(L.flags), 0u, 4, s) != hipSuccess) return fail(DM_ERR_DEVICE);
    // per dataset: validation, keys into the xs array, row statistics
    for (int32_t i = 0; i < count; ++i) {
        const MultiSet& q = m->sets[i];
        if (launch_fill_u32(h->at<uint32_t>(q.kmin), 0xffffffffu, (size_t)q.d, s) != hipSuccess ||
            launch_fill_u32(h->at<uint32_t>(q.kmax), 0u, (size_t)q.d, s) != hipSuccess)
            return fail(DM_ERR_DEVICE);
        // float coordinates are shifted by their centres (exact) before the
        // row sums and sorted values are formed from them
        float* c = q.is_int ? nullptr : h->at<float>(L.centre) + q.seg0;
        if (launch_prep_transpose(q.dtype, sets[i].X, q.n, q.d, h->at<uint32_t>(L.xs) + q.base, q.ld, nullptr,
                                  h->at<uint32_t>(q.kmin), h->at<uint32_t>(q.kmax), h->at<uint32_t>(L.flags),
                                  s) != hipSuccess ||
            (c && launch_centre(h->at<uint32_t>(q.kmin), h->at<uint32_t>(q.kmax), q.d, c, s) != hipSuccess) ||
            launch_row_stats(q.dtype, sets[i].X, q.n, q.d, h->ws + q.rowsum, h->ws + q.rownrm, s, 1, c) !=
                hipSuccess)
            return fail(DM_ERR_DEVICE);
    }
    // one segmented sort over every (dataset, coordinate) segment
    {
        std::vector<int64_t> koff, klen;
        std::vector<uint32_t> toff, tseg;
        std::vector<uint8_t> sint;
        uint32_t t = 0;
        for (const auto& q : m->sets) {
            const uint32_t tps = (uint32_t)((q.n + SORT_TILE - 1) / SORT_TILE);
            for (int32_t k = 0; k < q.d; ++k) {
                const uint32_t seg = (uint32_t)koff.size();
                koff.push_back(q.base + (int64_t)k * q.ld);
                klen.push_back(q.n);
                sint.push_back(q.is_int ? 1 : 0);
                toff.push_back(t);
                for (uint32_t j = 0; j < tps; ++j) tseg.push_back(seg);
                t += tps;
            }
        }
        toff.push_back(t);
        if (hipMemcpyAsync(h->ws + L.key_off, koff.data(), koff.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(h->ws + L.key_len, klen.data(), klen.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(h->ws + L.tile_off, toff.data(), toff.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(h->ws + L.tile_seg, tseg.data(), tseg.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(h->ws + L.seg_int, sint.data(), sint.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(DM_ERR_DEVICE);
        SegTables tb;
        tb.key_off = h->at<int64_t>(L.key_off);
        tb.key_len = h->at<int64_t>(L.key_len);
        tb.tile_off = h->at<uint32_t>(L.tile_off);
        tb.tile_seg = h->at<uint32_t>(L.tile_seg);
        tb.seg_int = h->at<uint8_t>(L.seg_int);
        tb.centre = h->at<float>(L.centre);
        tb.nseg = L.nseg;
        tb.ntiles = L.ntiles;
        uint32_t* K0 = h->at<uint32_t>(L.xs);
        uint32_t* V0 = h->at<uint32_t>(L.ids);
        uint32_t* K1 = h->at<uint32_t>(L.k1);
        uint32_t* V1 = h->at<uint32_t>(L.v1);
        uint32_t* perm = h->at<uint32_t>(L.perm);
        uint32_t* counts = h->at<uint32_t>(L.counts);
        const uint32_t* kin[4] = {K0, K1, K0, K1};
        const uint32_t* vin[4] = {nullptr, V1, V0, V1};
        uint32_t* kout[4] = {K1, K0, K1, K0};
        uint32_t* vout[4] = {V1, V0, V1, perm};
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 8 * pass;
            if (launch_sort_count(kin[pass], counts, tb, shift, s) != hipSuccess ||
                launch_sort_scan(counts, tb, s) != hipSuccess ||
                launch_sort_scatter(kin[pass], vin[pass], kout[pass], vout[pass], counts, tb, shift, pass == 0,
                                    pass == 3, false, s) != hipSuccess)
                return fail(DM_ERR_DEVICE);
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(DM_ERR_DEVICE);
    uint32_t flags = 0;
    if (hipMemcpy(&flags, h->ws + L.flags, 4, hipMemcpyDeviceToHost) != hipSuccess) return fail(DM_ERR_DEVICE);
    if (flags & FLAG_NONFINITE) return fail(DM_ERR_NONFINITE);
    if (flags & FLAG_INT_RANGE) return fail(DM_ERR_DTYPE);
    // descriptors (pinned mirror and device copy) and the totals block table
    const int nsets = count;
    if (hipHostMalloc((void**)&m->h_ds, (size_t)nsets * sizeof(MultiDs), hipHostMallocDefault) != hipSuccess)
        return fail(DM_ERR_NOMEM);
    m->d_ds = h->at<MultiDs>(L.ds);
    std::vector<uint32_t> blk;
    for (int32_t i = 0; i < nsets; ++i) {
        MultiSet& q = m->sets[i];
        std::vector<uint32_t> kmin(q.d), kmax(q.d);
        if (hipMemcpy(kmin.data(), h->ws + q.kmin, (size_t)q.d * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(kmax.data(), h->ws + q.kmax, (size_t)q.d * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(DM_ERR_DEVICE);
        double g = 0.0;
        for (int32_t k = 0; k < q.d; ++k) g += key_to_double(kmax[k], q.is_int) - key_to_double(kmin[k], q.is_int);
        q.guard = g;
        MultiDs& D = m->h_ds[i];
        std::memset(&D, 0, sizeof(D));
        D.perm = h->at<uint32_t>(L.perm) + q.base;
        D.xs = h->at<uint32_t>(L.xs) + q.base;
        D.rowsum = h->ws + q.rowsum;
        D.n = q.n;
        D.ld = q.ld;
        D.d = q.d;
        D.is_int = q.is_int ? 1 : 0;
        D.guard = g;
        D.tot_blk0 = (int64_t)blk.size();
        const int nb = (int)((q.n + multi_totals_rows() - 1) / multi_totals_rows());
        D.tot_nblk = nb;
        for (int j = 0; j < nb; ++j) blk.push_back((uint32_t)i);
    }
    m->nblk = (int)blk.size();
    if (m->nblk != L.nblk) return fail(DM_ERR_STATE);   // the layout counted the same blocks
    m->d_blk = h->at<uint32_t>(L.blk);
    if (hipMemcpy(m->d_blk, blk.data(), blk.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return fail(DM_ERR_DEVICE);
    h->last = s;
    *out = h;
    return DM_OK;
}

dm_status dm_matvec_multi(dm_handle* h, const void* const* Z, int32_t b, void* const* Out, void* stream) {
    if (!h || !Z || !Out || b < 1 || b > MAX_B) return DM_ERR_ARG;
    if (!h->multi) return DM_ERR_STATE;
    MultiState* m = h->multi;
    const int nsets = (int)m->sets.size();
    for (int i = 0; i < nsets; ++i) {
        if (!Z[i] || !Out[i]) return DM_ERR_ARG;
        const size_t zb = (size_t)m->sets[i].n * b * 4, ob = (size_t)m->sets[i].n * b * (m->sets[i].is_int ? 8 : 4);
        const char* zp = (const char*)Z[i];
        const char* op = (const char*)Out[i];
        if (zp < op + ob && op < zp + zb) return DM_ERR_ARG;
    }
    // 16-byte row accesses when every row of every dataset allows them; a
    // plan captured for the other choice (or another tile variant) is rebuilt
    bool vec = b % 4 == 0;
    for (int i = 0; i < nsets && vec; ++i) vec = ((uintptr_t)Z[i] % 16 == 0) && ((uintptr_t)Out[i] % 16 == 0);
    const int v = m->variant[log2_pad(b)];
    dm_status st;
    if ((m->plan.b != b || m->plan.vec != vec || m->plan.variant != v) && (st = build_plan(h, b, vec, v)) != DM_OK)
        return st;
    // refresh the pointer table only when it changes (the previous launch's
    // upload must have run before the pinned mirror is rewritten)
    bool same = true;
    for (int i = 0; i < nsets && same; ++i) same = m->h_ds[i].Z == Z[i] && m->h_ds[i].Out == Out[i];
    if (!same) {
        if (m->launched) DM_TRY(hipEventSynchronize(m->done));
        for (int i = 0; i < nsets; ++i) {
            m->h_ds[i].Z = Z[i];
            m->h_ds[i].Out = Out[i];
        }
    }
    hipStream_t s = (hipStream_t)stream;
    DM_TRY(hipGraphLaunch(m->plan.exec, s));
    DM_TRY(hipEventRecord(m->done, s));
    m->launched = true;
    h->last = s;
    return DM_OK;
}

int32_t dm_multi_variant_count(void) { return MULTI_VARIANTS; }

dm_status dm_set_variant_multi(dm_handle* h, int32_t b, int32_t variant) {
    if (!h || b < 1 || b > MAX_B || variant < 0 || variant >= MULTI_VARIANTS) return DM_ERR_ARG;
    if (!h->multi) return DM_ERR_STATE;
    h->multi->variant[log2_pad(b)] = (int8_t)variant;
    return DM_OK;
}

dm_status dm_get_variant_multi(dm_handle* h, int32_t b, int32_t* variant) {
    if (!h || !variant || b < 1 || b > MAX_B) return DM_ERR_ARG;
    if (!h->multi) return DM_ERR_STATE;
    *variant = h->multi->variant[log2_pad(b)];
    return DM_OK;
}

dm_status dm_tune_multi(dm_handle* h, const void* const* Z, int32_t b, void* const* Out, int32_t reps, void* stream,
                        int32_t* chosen, double* ms_per_query) {
    if (!h || !Z || !Out || b < 1 || b > MAX_B || reps < 1 || reps > 4096) return DM_ERR_ARG;
    if (!h->multi) return DM_ERR_STATE;
    MultiState* m = h->multi;
    hipStream_t s = (hipStream_t)stream;
    const int lg = log2_pad(b);
    const int8_t keep = m->variant[lg];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 1e300;
    int bestv = 0;
    // every variant: one untimed query (which builds its plan), then reps
    // timed graph launches on the caller's own right-hand sides
    auto run = [&]() -> dm_status {
        DM_TRY(hipEventCreate(&e0));
        DM_TRY(hipEventCreate(&e1));
        for (int v = 0; v < MULTI_VARIANTS; ++v) {
            m->variant[lg] = (int8_t)v;
            dm_status st = dm_matvec_multi(h, Z, b, Out, stream);
            if (st != DM_OK) return st;
            DM_TRY(hipEventRecord(e0, s));
            for (int i = 0; i < reps; ++i)
                if ((st = dm_matvec_multi(h, Z, b, Out, stream)) != DM_OK) return st;
            DM_TRY(hipEventRecord(e1, s));
            DM_TRY(hipEventSynchronize(e1));
            float t = 0.0f;
            DM_TRY(hipEventElapsedTime(&t, e0, e1));
            const double per = (double)t / reps;
            if (ms_per_query) ms_per_query[v] = per;
            if (per < best) {
                best = per;
                bestv = v;
            }
        }
        return DM_OK;
    };
    dm_status st = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != DM_OK) {
        m->variant[lg] = keep;
        return st;
    }
    m->variant[lg] = (int8_t)bestv;
    // leave the winner's plan captured (and Out holding its result)
    if ((st = dm_matvec_multi(h, Z, b, Out, stream)) != DM_OK) return st;
    if (chosen) *chosen = bestv;
    return DM_OK;
}

dm_status dm_multi_count(const dm_handle* h, int32_t* count) {
    if (!h || !count) return DM_ERR_ARG;
    if (!h->multi) return DM_ERR_STATE;
    *count = (int32_t)h->multi->sets.size();
    return DM_OK;
}

}  // extern "C"
