// tb_engine.hip -- plan, resident series store, workspaces, request queue and
// the C ABI of include/tb.h.  Host C++ on the HIP runtime; every step of the
// search itself runs in the kernels of tb_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "tb_internal.h"

using namespace tb;

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Host statistics of the threshold step (Sec. 2.1).  Whitened noise powers
// are unit exponentials, so a fold of h of them has the upper tail
// Q(h, x) = exp(-x) sum_{k<h} x^k / k!.
struct LogFactorials {
    double v[33];  // log k!, k = 0 .. 32 (h <= 16)
    LogFactorials()
    {
        for (int k = 0; k < 33; ++k) v[k] = std::lgamma((double)k + 1.0);
    }
};
const LogFactorials kLogFact;

// The sum is taken relative to its largest term, k* = min(h - 1, floor x),
// each neighbouring term from the last by the ratio x / k (or k / x), so only
// two logarithms are needed.
double log_q(int h, double x)
{
    if (x <= 0.0) return 0.0;
    const int ks = (int)std::min<double>(h - 1, std::floor(x));
    double acc = 1.0, r = 1.0;
    for (int k = ks; k >= 1; --k) {
        r *= (double)k / x;
        acc += r;
    }
    r = 1.0;
    for (int k = ks + 1; k < h; ++k) {
        r *= x / (double)k;
        acc += r;
    }
    return -x + ks * std::log(x) - kLogFact.v[ks] + std::log(acc);
}

const double kHalfLog2Pi = 0.5 * std::log(2.0 * kPi);
const double kRsqrt2 = 1.0 / std::sqrt(2.0);

// log of the one-sided Gaussian tail; from z = 37 on (where erfc nears the
// bottom of the double range) via the continued fraction of the Mills ratio.
double log_gauss_sf(double z)
{
    if (z < 37.0) return std::log(0.5 * std::erfc(z * kRsqrt2));
    double f = z;
    for (int k = 80; k >= 1; --k) f = z + (double)k / f;
    return -0.5 * z * z - kHalfLog2Pi - std::log(f);
}

// Threshold x with log Q(h, x) = log_gauss_sf(sigma): bracket, then
// Newton steps kept inside the bracket.
double fold_threshold(int h, double sigma)
{
    double target = log_gauss_sf(sigma);
    double lo = 0.0, hi = 8.0;
    while (log_q(h, hi) > target) {
        lo = hi;
        hi *= 2.0;
    }
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double g = log_q(h, x) - target;
        if (g > 0) lo = x; else hi = x;
        double dg = -std::exp((h - 1) * std::log(x) - x - std::lgamma((double)h) - log_q(h, x));
        double nx = x - g / dg;
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        if (std::fabs(nx - x) < 1e-13 * std::max(1.0, x)) {
            x = nx;
            break;
        }
        x = nx;
    }
    return x;
}

// ---------------------------------------------------------------------------
struct SeriesRec {
    int64_t n = 0;
    double tsamp = 0;
    float* d = nullptr;
    size_t bytes = 0;     // everything the series holds
    float* fac = nullptr; // whitened once: factors ln2 / m(k), M + 1 floats; nullptr = per template
    float* med = nullptr; // and the series' block medians (same allocation)
    int2* zap = nullptr;  // birdie bin ranges [x, y], sorted and disjoint (own allocation)
    int nzap = 0;
    size_t zap_bytes = 0;
};

struct GeoRec {
    Geometry g;
    size_t bytes = 0;
};

struct SlotRec {
    Slots s;
    size_t bytes = 0;
};

void free_slots(Slots& s)
{
    hipFree(s.Y);
    hipFree(s.P);
    hipFree(s.Q);
    hipFree(s.med);
    hipFree(s.poly);
    hipFree(s.pok);
    s = Slots();
}

struct Lane {
    hipStream_t stream = nullptr;
    bool own = false;
    std::map<int, SlotRec> slots;  // workspaces by log2 n
    double pending = 0;            // queued work of unsettled requests (template-samples)
};

struct Req {
    int lane = 0;         // primary lane: request memory and the completion event live on its stream
    double work = 0;      // templates x samples, for lane balancing
    bool settled = false; // completion already subtracted from the lanes' pending work
    std::vector<std::pair<int, double>> parts;  // (lane, work) of every lane the waves run on
    std::vector<hipEvent_t> joins;              // primary ready / helper lanes done
    int32_t series = -1;
    uint32_t count = 0, first = 0;
    uint64_t cap = 0;
    int64_t n = 0;
    double tsamp = 0;
    char* dmem = nullptr;       // templates (device copy), prepared templates, counter, ring
    size_t dmem_size = 0;
    tb_template* h_t = nullptr; // pinned host copy
    size_t h_t_size = 0;
    size_t bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool fetched = false;
    uint32_t total = 0;
    std::vector<tb_candidate> cands;
};

}  // namespace

struct tb_plan_s {
    tb_config cfg;
    hipStream_t stream = nullptr;  // lane 0: loads, inspection, utilities
    hipStream_t copy_stream = nullptr;
    std::vector<Lane> lanes;       // requests spread over these streams
    std::mutex mu;
    std::map<int32_t, SeriesRec> series;
    std::map<int, GeoRec> geo;     // by log2 n
    std::map<int, std::pair<int, int>> shape;  // per log2 n: (tile points, templates per wave) set by tb_set_shape
    std::map<int64_t, Req> reqs;
    int32_t next_series = 0;
    int64_t next_req = 1;
    uint64_t held = 0;
    double thr[5] = {0, 0, 0, 0, 0};
    double* d_partial = nullptr;
    // Request buffers kept for reuse after tb_release (device slabs and pinned
    // template copies, by size): steady-state submits allocate nothing.
    std::multimap<size_t, char*> dev_pool;
    std::multimap<size_t, tb_template*> pin_pool;
    uint32_t prof_every = 0;                           // time every k-th wave; 0 = off
    uint64_t prof_wave = 0;                            // waves queued since profiling started
    std::vector<Marks> prof_events;                    // marks of every timed wave
    uint64_t prof_templates = 0;
};

namespace {

#define TB_TRY(call)                                   \
    do {                                               \
        if ((call) != hipSuccess) return TB_ERR_DEVICE; \
    } while (0)

bool pow2(uint64_t v) { return v && !(v & (v - 1)); }
int ilog2(uint64_t v)
{
    int l = 0;
    while ((1ull << l) < v) ++l;
    return l;
}

tb_status reserve(tb_plan_t p, size_t bytes)
{
    if (p->cfg.hbm_budget_bytes && p->held + bytes > p->cfg.hbm_budget_bytes) return TB_ERR_BUDGET;
    p->held += bytes;
    return TB_OK;
}

tb_status upload_table(std::vector<float2>& h, float2** d, size_t* bytes)
{
    size_t b = h.size() * sizeof(float2);
    if (hipMalloc(d, b) != hipSuccess) return TB_ERR_OOM;
    TB_TRY(hipMemcpy(*d, h.data(), b, hipMemcpyHostToDevice));
    *bytes += b;
    return TB_OK;
}

// exp(-2 pi i r num / den) for r < count, in FP64 then rounded.
std::vector<float2> twiddles(int64_t count, double num, double den)
{
    std::vector<float2> t((size_t)count);
    for (int64_t r = 0; r < count; ++r) {
        double a = -2.0 * kPi * ((double)r * num) / den;
        t[(size_t)r] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    return t;
}

// Radix-16 stage twiddles, in the order the kernels index them: for strides
// NS = 2..16 a record of W_{16 NS}^{r k}, r = 1..15, per k < NS (450 entries
// in all, zero-padded), then for NS = 32..ns_max the powers W_{16 NS}^i,
// i < 16 NS (the table of a longer transform extends that of a shorter one).
std::vector<float2> stage_twiddles(int ns_max)
{
    auto w = [](double num, double den) {
        double a = -2.0 * kPi * num / den;
        return make_float2((float)std::cos(a), (float)std::sin(a));
    };
    std::vector<float2> t;
    for (int ns = 2; ns <= 16; ns *= 2)
        for (int k = 0; k < ns; ++k)
            for (int r = 1; r < 16; ++r) t.push_back(ns <= ns_max ? w((double)(r * k), 16.0 * ns) : make_float2(0, 0));
    for (int ns = 32; ns <= ns_max; ns *= 2)
        for (int i = 0; i < 16 * ns; ++i) t.push_back(w((double)i, 16.0 * ns));
    return t;
}

// Harmonic-sum tile order for a grid of ntile rounded up to a multiple of 8
// workgroups (workgroup x runs on XCD x % 8): binary subtrees of tiles
// {r, 2r, 2r+1, 4r, ...}, r in [2^a, 2^(a+1)) with about 64 tiles per tree,
// go whole to one XCD in breadth-first order (a tile's parent before it);
// tiles below 2^a are spread round robin.
std::vector<int32_t> harmsum_order(int ntile)
{
    const int X = 8;
    std::vector<std::vector<int32_t>> q(X);
    int a = 3;  // at least 8 roots
    while ((2 << a) * 64 <= ntile) ++a;  // roots [2^a, 2^(a+1)): trees of ~64 tiles (best of 16..256)
    const int r0 = 1 << a;
    int next = 0;
    for (int r = r0; r < 2 * r0 && r < ntile; ++r) {
        std::vector<int32_t>& dst = q[next];
        next = (next + 1) % X;
        for (int64_t lo = r, width = 1; lo < ntile; lo *= 2, width *= 2)
            for (int64_t t = lo; t < lo + width && t < ntile; ++t) dst.push_back((int32_t)t);
    }
    for (int t = 0; t < r0 && t < ntile; ++t) {
        // the shortest queue takes the next low tile
        int best = 0;
        for (int c = 1; c < X; ++c)
            if (q[c].size() < q[best].size()) best = c;
        q[best].push_back(t);
    }
    size_t longest = 0;
    for (auto& v : q) longest = std::max(longest, v.size());
    std::vector<int32_t> tile_of(longest * X, -1);
    for (int c = 0; c < X; ++c)
        for (size_t k = 0; k < q[c].size(); ++k) tile_of[k * X + c] = q[c][k];
    return tile_of;
}

tb_status get_geometry(tb_plan_t p, int log2n, Geometry** out)
{
    auto it = p->geo.find(log2n);
    if (it != p->geo.end()) {
        *out = &it->second.g;
        return TB_OK;
    }
    GeoRec rec;
    Geometry& g = rec.g;
    g.log2n = log2n;
    g.n = (int64_t)1 << log2n;
    g.M = g.n / 2;
    // 8192-point tiles (two workgroups per CU) up to 2^23 samples; at 2^24 they
    // would leave pass 2 with 8-column workgroups and 32-byte reads
    g.TE = p->cfg.tile_points ? (int)p->cfg.tile_points : (g.M >= ((int64_t)1 << 23) ? 16384 : 8192);
    auto sh = p->shape.find(log2n);
    if (sh != p->shape.end() && sh->second.first) g.TE = sh->second.first;
    const int64_t TE = std::min<int64_t>(g.TE, g.M);
    g.R = (int)std::max<int64_t>(16, g.M / g.TE);
    g.S = (int)(g.M / g.R);
    g.C1 = (int)(TE / g.S);
    g.lgR = ilog2((uint64_t)g.R);
    // rows of 2R samples: enough for a delay swing of n/8 samples, at most
    // 2^PAD_REACH_LOG2, plus two for rounding
    g.P = (int)(std::min<int64_t>(g.n / 8, (int64_t)1 << PAD_REACH_LOG2) / (2 * g.R)) + 2;
    // pass-2 workgroups take at most 8192 points (16 columns of 512 at 2^24):
    // with one column per pass-1 workgroup any column count divides the
    // exchange evenly, and the 8192-point shape runs two workgroups per CU
    g.D2 = (int)((TE > 8192 && g.C1 == 1 ? 8192 : TE) / g.R);
    g.W = (int)p->cfg.whiten_window;
    g.nblk = (int)((g.M + g.W - 1) / g.W);
    g.htile = harmsum_tile();
    int64_t hi = std::max<int64_t>(1, g.M >> TW_LO_BITS);
    std::vector<float2> v;
    tb_status st;
    {
        std::vector<int32_t> order = harmsum_order((int)((g.M + 1 + g.htile - 1) / g.htile));
        size_t b = order.size() * sizeof(int32_t);
        g.hgrid = (int)order.size();
        if (hipMalloc(&g.tile_of, b) != hipSuccess) return TB_ERR_OOM;
        TB_TRY(hipMemcpy(g.tile_of, order.data(), b, hipMemcpyHostToDevice));
        rec.bytes += b;
    }
    v = stage_twiddles(std::max(2, std::max(g.S, g.R) / 16));
    if ((st = upload_table(v, &g.twst, &rec.bytes))) return st;
    v = twiddles(1 << TW_LO_BITS, 1.0, (double)g.M);
    if ((st = upload_table(v, &g.twM_lo, &rec.bytes))) return st;
    v = twiddles(hi, (double)(1 << TW_LO_BITS), (double)g.M);
    if ((st = upload_table(v, &g.twM_hi, &rec.bytes))) return st;
    v = twiddles(1 << TW_LO_BITS, 1.0, 2.0 * (double)g.M);
    if ((st = upload_table(v, &g.tw2M_lo, &rec.bytes))) return st;
    v = twiddles(hi, (double)(1 << TW_LO_BITS), 2.0 * (double)g.M);
    if ((st = upload_table(v, &g.tw2M_hi, &rec.bytes))) return st;
    p->held += rec.bytes;
    auto ins = p->geo.emplace(log2n, rec);
    *out = &ins.first->second.g;
    return TB_OK;
}

void free_geometry(GeoRec& r)
{
    hipFree(r.g.twst);
    hipFree(r.g.tile_of);
    hipFree(r.g.twM_lo);
    hipFree(r.g.twM_hi);
    hipFree(r.g.tw2M_lo);
    hipFree(r.g.tw2M_hi);
}

int default_batch(const tb_plan_t p, int64_t M)
{
    auto sh = p->shape.find(ilog2((uint64_t)M) + 1);
    if (sh != p->shape.end() && sh->second.second) return sh->second.second;
    if (p->cfg.batch_templates) return (int)p->cfg.batch_templates;
    int64_t b = ((int64_t)1 << 28) / M;  // 2^28 bins in flight: 64 templates at 2^23 samples
    return (int)std::min<int64_t>(256, std::max<int64_t>(4, b));
}

tb_status get_slots(tb_plan_t p, int lane, const Geometry& g, Slots** out)
{
    auto& slots = p->lanes[lane].slots;
    auto it = slots.find(g.log2n);
    if (it != slots.end()) {
        *out = &it->second.s;
        return TB_OK;
    }
    SlotRec rec;
    Slots& s = rec.s;
    s.B = default_batch(p, g.M);
    // passes 1 and 2 in groups whose exchange buffer (8M bytes per template)
    // stays within about 128 MiB, so that pass 2 reads it from the cache
    s.BY = (int)std::max<int64_t>(1, std::min<int64_t>(s.B, ((int64_t)1 << 24) / g.M));
    s.y_stride = (size_t)g.M;
    s.p_stride = ((size_t)g.M + 1 + 63) & ~(size_t)63;
    s.med_stride = ((size_t)g.nblk + 63) & ~(size_t)63;
    s.poly_stride = (size_t)std::min<int64_t>(g.TE, g.M) / 8;
    size_t by = sizeof(float2) * s.y_stride * s.BY, bp = sizeof(float) * s.p_stride * s.B,
           bm = sizeof(float) * s.med_stride * s.B, bq = sizeof(ChunkPoly) * s.poly_stride * s.B,
           bk = sizeof(int32_t) * (size_t)s.B;
    rec.bytes = by + 2 * bp + bm + bq + bk;
    tb_status st = reserve(p, rec.bytes);
    if (st) return st;
    if (hipMalloc(&s.Y, by) != hipSuccess || hipMalloc(&s.P, bp) != hipSuccess || hipMalloc(&s.Q, bp) != hipSuccess ||
        hipMalloc(&s.med, bm) != hipSuccess || hipMalloc(&s.poly, bq) != hipSuccess ||
        hipMalloc(&s.pok, bk) != hipSuccess) {
        free_slots(s);
        p->held -= rec.bytes;
        return TB_ERR_OOM;
    }
    auto ins = slots.emplace(g.log2n, rec);
    *out = &ins.first->second.s;
    return TB_OK;
}

PeakParams peak_params(tb_plan_t p, int64_t n, double tsamp, uint32_t series_id, uint32_t first, uint64_t cap)
{
    PeakParams pp;
    std::memset(&pp, 0, sizeof(pp));
    int64_t M = n / 2;
    double T = (double)n * tsamp;
    int64_t kmin = (int64_t)std::ceil(p->cfg.fmin_hz * T);
    if (kmin < 1) kmin = 1;
    pp.nfold = ilog2(p->cfg.harm_max) + 1;
    for (int l = 0; l < 5; ++l) {
        int64_t h = (int64_t)1 << l;
        pp.thr[l] = (float)p->thr[l];
        pp.klo[l] = (int32_t)std::min<int64_t>(M + 1, h * kmin);
        int64_t khi = M;
        if (p->cfg.fmax_hz > 0.0) khi = std::min<int64_t>(M, (int64_t)std::floor((double)h * p->cfg.fmax_hz * T));
        pp.khi[l] = (int32_t)std::max<int64_t>(-1, khi);
    }
    pp.series_id = series_id;
    pp.first_template_id = first;
    pp.capacity = (uint32_t)std::min<uint64_t>(cap, 0xffffffffull);
    return pp;
}

int delay_model(const tb_plan_t p) { return (p->cfg.flags & TB_DELAY_SERIES) ? 1 : 0; }

// Sample indices stay 32-bit: the delay swing may not exceed 2^29 samples.
// |F| <= 1 + e for the BT delay, e + sum |C_k| + |S_k| for the series.
bool delay_fits(const tb_plan_t p, const tb_template& t, double tsamp)
{
    double bound = 1.0 + t.ecc;
    if (delay_model(p)) {
        double C[8], S[8];
        series_coefficients(t.ecc, C, S);
        bound = t.ecc;
        for (int k = 0; k < 8; ++k) bound += std::fabs(C[k]) + std::fabs(S[k]);
    }
    return 2.0 * t.tau_lts * bound / tsamp <= (double)(1 << 29);
}

bool valid_template(const tb_template& t)
{
    return std::isfinite(t.porb_s) && std::isfinite(t.tau_lts) && std::isfinite(t.alpha_rad) &&
           std::isfinite(t.ecc) && std::isfinite(t.omega_rad) && t.porb_s > 0.0 && t.tau_lts >= 0.0 &&
           t.ecc >= 0.0 && t.ecc < 1.0;
}

// Request buffers: a pooled one of at least `need` bytes and at most twice
// that, else a new one of `need` rounded up to 1 MiB (device) or 4 KiB
// (pinned host).  Returned buffers are kept, up to kPoolKeep of each kind;
// the plan frees them in tb_destroy.  Only buffers of requests whose device
// work has completed are returned.
constexpr size_t kPoolKeep = 32;

template <class T>
T* pool_take(std::multimap<size_t, T*>& pool, size_t need, size_t* got)
{
    auto it = pool.lower_bound(need);
    if (it == pool.end() || it->first > 2 * need) return nullptr;
    T* ptr = it->second;
    *got = it->first;
    pool.erase(it);
    return ptr;
}

template <class T, class F>
void pool_give(std::multimap<size_t, T*>& pool, size_t bytes, T* ptr, F release)
{
    if (!ptr) return;
    pool.emplace(bytes, ptr);
    if (pool.size() > kPoolKeep) {
        auto it = pool.begin();  // the smallest goes
        release(it->second);
        pool.erase(it);
    }
}

char* take_device(tb_plan_t p, size_t need, size_t* got)
{
    if (char* d = pool_take(p->dev_pool, need, got)) return d;
    const size_t size = (need + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
    char* d = nullptr;
    if (hipMalloc((void**)&d, size) != hipSuccess) {
        // memory may sit in the pool: give it back and try once more
        for (auto& kv : p->dev_pool) hipFree(kv.second);
        p->dev_pool.clear();
        if (hipMalloc((void**)&d, size) != hipSuccess) return nullptr;
    }
    *got = size;
    return d;
}

tb_template* take_pinned(tb_plan_t p, size_t need, size_t* got)
{
    if (tb_template* h = pool_take(p->pin_pool, need, got)) return h;
    const size_t size = (need + 4095) & ~(size_t)4095;
    void* h = nullptr;
    if (hipHostMalloc(&h, size, hipHostMallocDefault) != hipSuccess) return nullptr;
    *got = size;
    return (tb_template*)h;
}

void free_request(tb_plan_t p, Req& r)
{
    if (r.ev0) hipEventDestroy(r.ev0);
    if (r.ev1) hipEventDestroy(r.ev1);
    for (hipEvent_t e : r.joins) hipEventDestroy(e);
    r.joins.clear();
    pool_give(p->dev_pool, r.dmem_size, r.dmem, [](char* d) { hipFree(d); });
    pool_give(p->pin_pool, r.h_t_size, r.h_t, [](tb_template* h) { hipHostFree(h); });
    r.dmem = nullptr;
    r.h_t = nullptr;
}

struct ReqLayout {
    size_t off_t, off_tm, off_cnt, off_ring, total;
};

ReqLayout req_layout(uint32_t count, uint64_t cap)
{
    ReqLayout L;
    L.off_t = 0;
    L.off_tm = ((size_t)count * sizeof(tb_template) + 255) & ~(size_t)255;
    L.off_cnt = L.off_tm + (((size_t)count * sizeof(TmplDev) + 255) & ~(size_t)255);
    L.off_ring = L.off_cnt + 256;
    L.total = L.off_ring + (size_t)cap * sizeof(uint4);
    return L;
}

// Queue the kernels of all templates of a request, wave by wave; wave i goes
// to workspace i mod (number of workspaces) on that workspace's stream.
struct Crew {
    std::vector<hipStream_t> streams;
    std::vector<Slots*> slots;
};

tb_status enqueue(tb_plan_t p, const Crew& crew, const SeriesRec& sr, Geometry* g, const TmplDev* d_tm,
                  uint32_t count, const PeakParams& pp, uint4* ring, uint32_t* counter, const Inspect& ins)
{
    const size_t nc = crew.streams.size();
    size_t wave = 0;
    for (uint32_t w0 = 0; w0 < count; ++wave) {
        Slots* ws = crew.slots[wave % nc];
        hipStream_t stream = crew.streams[wave % nc];
        int nslots = (int)std::min<uint32_t>((uint32_t)ws->B, count - w0);
        Marks* marks = nullptr;
        if (p->prof_every && p->prof_wave++ % p->prof_every == 0) {
            p->prof_events.emplace_back();
            marks = &p->prof_events.back();
            p->prof_templates += (uint64_t)nslots;
        }
        if (launch_wave(*g, sr.d, sr.tsamp, d_tm, (int)w0, nslots, *ws, sr.fac, sr.zap, sr.nzap, pp, ring, counter,
                        ins, stream,
                        marks) !=
            hipSuccess)
            return TB_ERR_DEVICE;
        w0 += (uint32_t)nslots;
    }
    return TB_OK;
}

// Subtracts finished requests from their lane's pending work.
void settle(tb_plan_t p)
{
    for (auto& kv : p->reqs) {
        Req& r = kv.second;
        if (!r.settled && hipEventQuery(r.ev1) == hipSuccess) {
            for (auto& pw : r.parts) p->lanes[pw.first].pending -= pw.second;
            r.settled = true;
        }
    }
}

// The lane with the least queued work.
int pick_lane(tb_plan_t p)
{
    settle(p);
    int best = 0;
    for (int l = 1; l < (int)p->lanes.size(); ++l)
        if (p->lanes[l].pending < p->lanes[best].pending) best = l;
    return best;
}

hipError_t sync_lanes(tb_plan_t p)
{
    hipError_t e = hipSuccess;
    for (auto& L : p->lanes) {
        hipError_t f = hipStreamSynchronize(L.stream);
        if (e == hipSuccess) e = f;
    }
    return e;
}

// A ring record after launch_significance, {template, bin | log2 h << 28,
// sigma, S}, as the candidate of series sid with its fundamental frequency
// k / (h T).
void to_candidate(const uint4& q, uint32_t sid, double T, tb_candidate& c)
{
    std::memset(&c, 0, sizeof(c));
    c.series_id = sid;
    c.template_id = q.x;
    c.bin = q.y & 0x0fffffffu;
    c.log2_harm = (uint8_t)(q.y >> 28);
    std::memcpy(&c.sigma, &q.z, sizeof(float));
    std::memcpy(&c.power, &q.w, sizeof(float));
    c.freq_hz = (double)c.bin / ((double)(1 << c.log2_harm) * T);
}

void sort_candidates(tb_candidate* c, size_t n)
{
    std::sort(c, c + n, [](const tb_candidate& a, const tb_candidate& b) {
        if (a.series_id != b.series_id) return a.series_id < b.series_id;
        if (a.template_id != b.template_id) return a.template_id < b.template_id;
        if (a.log2_harm != b.log2_harm) return a.log2_harm < b.log2_harm;
        return a.bin < b.bin;
    });
}

// One request's records (one series) in candidate order: template, fold, bin.
void sort_records(std::vector<uint4>& raw)
{
    std::sort(raw.begin(), raw.end(), [](const uint4& a, const uint4& b) {
        if (a.x != b.x) return a.x < b.x;
        if ((a.y >> 28) != (b.y >> 28)) return (a.y >> 28) < (b.y >> 28);
        return (a.y & 0x0fffffffu) < (b.y & 0x0fffffffu);
    });
}

tb_status fetch(tb_plan_t p, Req& r)
{
    if (r.fetched) return TB_OK;
    ReqLayout L = req_layout(r.count, r.cap);
    uint32_t total = 0;
    TB_TRY(hipMemcpyAsync(&total, r.dmem + L.off_cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, p->copy_stream));
    TB_TRY(hipStreamSynchronize(p->copy_stream));
    uint64_t keep = std::min<uint64_t>(total, r.cap);
    std::vector<uint4> raw((size_t)keep);
    if (keep) {
        TB_TRY(hipMemcpyAsync(raw.data(), r.dmem + L.off_ring, keep * sizeof(uint4), hipMemcpyDeviceToHost,
                              p->copy_stream));
        TB_TRY(hipStreamSynchronize(p->copy_stream));
    }
    const double T = (double)r.n * r.tsamp;
    sort_records(raw);
    r.cands.resize((size_t)keep);
    for (size_t i = 0; i < raw.size(); ++i) to_candidate(raw[i], (uint32_t)r.series, T, r.cands[i]);
    r.total = total;
    r.fetched = true;
    return TB_OK;
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free search (tb_search_templates_noalloc).
// The library's code object is loaded on every GPU it runs on, so each GPU
// holds its own copy of this array, at its own address, until the process
// ends.  In host code the name is only a stand-in: the device address on a
// GPU comes from hipGetSymbolAddress with that GPU current (done once per
// device, when its first plan is created) and is the only thing host code
// hands to kernels or copies.
static __device__ __align__(256) unsigned char scratch[TB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of the scratch on device dev, which must be current.
hipError_t scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = (char*)ptr;
    return hipSuccess;
}

char* scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

// Request part (templates, prepared templates, counter, ring), then a
// workspace for B templates per wave laid out as get_slots lays out its own;
// B is the plan's wave size, halved until everything fits the scratch.
struct ScratchLayout {
    ReqLayout req;
    Slots ws;
    size_t off_y = 0, off_p = 0, off_w = 0, off_m = 0, off_q = 0, off_k = 0, total = 0;
};

bool scratch_layout(const tb_plan_t p, const Geometry& g, uint32_t count, uint64_t cap, ScratchLayout* out)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    ScratchLayout L;
    L.req = req_layout(count, cap);
    for (int B = default_batch(p, g.M);; B = std::max(1, B / 2)) {
        Slots& s = L.ws;
        s.B = B;
        s.BY = (int)std::max<int64_t>(1, std::min<int64_t>(B, ((int64_t)1 << 24) / g.M));
        s.y_stride = (size_t)g.M;
        s.p_stride = ((size_t)g.M + 1 + 63) & ~(size_t)63;
        s.med_stride = ((size_t)g.nblk + 63) & ~(size_t)63;
        s.poly_stride = (size_t)std::min<int64_t>(g.TE, g.M) / 8;
        L.off_y = al(L.req.total);
        L.off_p = L.off_y + al(sizeof(float2) * s.y_stride * s.BY);
        L.off_w = L.off_p + al(sizeof(float) * s.p_stride * s.B);
        L.off_m = L.off_w + al(sizeof(float) * s.p_stride * s.B);
        L.off_q = L.off_m + al(sizeof(float) * s.med_stride * s.B);
        L.off_k = L.off_q + al(sizeof(ChunkPoly) * s.poly_stride * s.B);
        L.total = L.off_k + al(sizeof(int32_t) * (size_t)s.B);
        if (L.total <= (size_t)TB_NOALLOC_SCRATCH_BYTES) {
            *out = L;
            return true;
        }
        if (B == 1) return false;
    }
}

}  // namespace

extern "C" {

void tb_default_config(tb_config* c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->max_log2n = 24;
    c->harm_max = 16;
    c->whiten_window = 4096;
    c->batch_templates = 0;
    c->threshold_sigma = 6.0;
    c->fmin_hz = 1.0;
    c->fmax_hz = 0.0;
    c->hbm_budget_bytes = 0;
    c->ring_capacity = 1u << 20;
    c->stream = nullptr;
    c->device = 0;
    c->lanes = 1;
    c->flags = 0;
    c->tile_points = 0;
}

const char* tb_strerror(tb_status s)
{
    switch (s) {
    case TB_OK: return "ok";
    case TB_ERR_INVALID_ARG: return "invalid argument";
    case TB_ERR_OOM: return "out of memory";
    case TB_ERR_BUDGET: return "HBM budget exceeded";
    case TB_ERR_DEVICE: return "HIP runtime error";
    case TB_ERR_OVERFLOW: return "candidate ring overflowed";
    case TB_ERR_NOT_READY: return "not ready";
    case TB_ERR_UNKNOWN_ID: return "unknown id";
    case TB_ERR_TOO_LARGE: return "does not fit the fixed scratch of the allocation-free search";
    }
    return "unknown status";
}

tb_status tb_plan(const tb_config* cfg, tb_plan_t* out)
{
    if (!cfg || !out) return TB_ERR_INVALID_ARG;
    *out = nullptr;
    const tb_config& c = *cfg;
    if (c.max_log2n < 10 || c.max_log2n > 24) return TB_ERR_INVALID_ARG;
    if (c.harm_max != 1 && c.harm_max != 2 && c.harm_max != 4 && c.harm_max != 8 && c.harm_max != 16)
        return TB_ERR_INVALID_ARG;
    if (c.whiten_window < 1 || c.whiten_window > 8192) return TB_ERR_INVALID_ARG;
    if (!std::isfinite(c.threshold_sigma) || !std::isfinite(c.fmin_hz) || !std::isfinite(c.fmax_hz) ||
        c.fmin_hz < 0.0 || c.fmax_hz < 0.0)
        return TB_ERR_INVALID_ARG;
    if (c.ring_capacity == 0 || c.ring_capacity > 0xffffffffull || c.batch_templates > 4096 ||
        (c.flags & ~(uint32_t)TB_DELAY_SERIES) ||
        (c.tile_points != 0 && c.tile_points != 8192 && c.tile_points != 16384) || c.lanes < 1 || c.lanes > 16)
        return TB_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c.device < 0 || c.device >= ndev) return TB_ERR_DEVICE;
    if (hipSetDevice(c.device) != hipSuccess) return TB_ERR_DEVICE;
    // the allocation-free search's scratch on this device
    if (scratch_setup(c.device) != hipSuccess) return TB_ERR_DEVICE;
    tb_plan_t p = new (std::nothrow) tb_plan_s();
    if (!p) return TB_ERR_OOM;
    p->cfg = c;
    p->lanes.resize(c.lanes);
    bool ok = true;
    for (uint32_t l = 0; l < c.lanes && ok; ++l) {
        Lane& L = p->lanes[l];
        if (l == 0 && c.stream) {
            L.stream = (hipStream_t)c.stream;
        } else {
            ok = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
            L.own = ok;
        }
    }
    if (ok) p->stream = p->lanes[0].stream;
    if (!ok || hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&p->d_partial, sizeof(double) * 1040) != hipSuccess) {
        for (auto& L : p->lanes)
            if (L.own) hipStreamDestroy(L.stream);
        if (p->copy_stream) hipStreamDestroy(p->copy_stream);
        delete p;
        return TB_ERR_DEVICE;
    }
    for (int l = 0; l < 5; ++l) p->thr[l] = (1u << l) <= c.harm_max ? fold_threshold(1 << l, c.threshold_sigma) : 0.0;
    *out = p;
    return TB_OK;
}

tb_status tb_destroy(tb_plan_t p)
{
    if (!p) return TB_OK;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        hipSetDevice(p->cfg.device);
        sync_lanes(p);
        for (auto& kv : p->reqs) free_request(p, kv.second);
        sync_lanes(p);
        for (auto& kv : p->dev_pool) hipFree(kv.second);
        for (auto& kv : p->pin_pool) hipHostFree(kv.second);
        for (auto& kv : p->series) {
            hipFree(kv.second.d);
            hipFree(kv.second.zap);
        }
        for (auto& L : p->lanes)
            for (auto& kv : L.slots) free_slots(kv.second.s);
        for (auto& kv : p->geo) free_geometry(kv.second);
        for (auto& v : p->prof_events)
            for (auto& m : v) hipEventDestroy(m.second);
        hipFree(p->d_partial);
        hipStreamDestroy(p->copy_stream);
        for (auto& L : p->lanes)
            if (L.own) hipStreamDestroy(L.stream);
    }
    delete p;
    return TB_OK;
}

tb_status tb_load_series(tb_plan_t p, const float* data, uint64_t n, double tsamp, uint32_t flags, int32_t* id)
{
    const uint32_t mem = flags & ~(uint32_t)TB_SERIES_WHITENING;
    const bool once = (flags & TB_SERIES_WHITENING) != 0;
    if (!p || !data || !id || !pow2(n) || n < 1024 || n > (1ull << p->cfg.max_log2n) || !(tsamp > 0.0) ||
        !std::isfinite(tsamp) || (mem != TB_MEM_HOST && mem != TB_MEM_DEVICE))
        return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    TB_TRY(hipSetDevice(p->cfg.device));
    if (p->next_series >= (1 << 24)) return TB_ERR_INVALID_ARG;
    Geometry* g = nullptr;
    tb_status st = get_geometry(p, ilog2(n), &g);
    if (st) return st;
    Slots* ws = nullptr;
    if (once && (st = get_slots(p, 0, *g, &ws))) return st;
    SeriesRec r;
    r.n = (int64_t)n;
    r.tsamp = tsamp;
    const size_t series_bytes = sizeof(float) * series_floats(*g);
    const size_t fac_floats = ((size_t)g->M + 1 + 63) & ~(size_t)63;
    r.bytes = series_bytes + (once ? sizeof(float) * (fac_floats + (size_t)g->nblk) : 0);
    if ((st = reserve(p, r.bytes))) return st;
    // one allocation: series (and padding), then factors and medians
    char* mem_d = nullptr;
    if (hipMalloc(&mem_d, r.bytes) != hipSuccess) {
        p->held -= r.bytes;
        return TB_ERR_OOM;
    }
    r.d = (float*)mem_d;
    if (once) {
        r.fac = (float*)(mem_d + series_bytes);
        r.med = r.fac + fac_floats;
    }
    // staging: [0, n) raw copy (host input), [n, 2n) mean-removed natural
    // order, then a template without orbit for the series levels
    float* staging = nullptr;
    const size_t tmpl_off = ((2 * sizeof(float) * n) + 255) & ~(size_t)255;
    if (hipMalloc(&staging, tmpl_off + 256 + sizeof(TmplDev)) != hipSuccess) {
        hipFree(r.d);
        p->held -= r.bytes;
        return TB_ERR_OOM;
    }
    const float* src = data;
    hipError_t e = hipSuccess;
    if (mem == TB_MEM_HOST) {
        e = hipMemcpyAsync(staging, data, sizeof(float) * n, hipMemcpyHostToDevice, p->stream);
        src = staging;
    }
    if (e == hipSuccess) e = launch_mean_subtract(src, staging + n, r.n, p->d_partial, p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(r.d, 0, series_bytes, p->stream);  // the zero rows
    if (e == hipSuccess) e = launch_tile_series(*g, staging + n, r.d, p->stream);
    if (e == hipSuccess && once) {
        // tau = 0: the demodulation reads every sample where it is
        static const tb_template still = {1.0, 0.0, 0.0, 0.0, 0.0};
        tb_template* d_t = (tb_template*)((char*)staging + tmpl_off);
        TmplDev* d_tm = (TmplDev*)((char*)staging + tmpl_off + 256);
        e = hipMemcpyAsync(d_t, &still, sizeof(still), hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) e = launch_template_prep(d_t, 1, d_tm, 0, p->stream);
        if (e == hipSuccess) e = launch_series_levels(*g, r.d, tsamp, d_tm, *ws, r.med, r.fac, p->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    hipFree(staging);
    if (e != hipSuccess) {
        hipFree(r.d);
        p->held -= r.bytes;
        return TB_ERR_DEVICE;
    }
    *id = p->next_series++;
    p->series.emplace(*id, r);
    return TB_OK;
}

tb_status tb_unload_series(tb_plan_t p, int32_t id)
{
    if (!p) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->series.find(id);
    if (it == p->series.end()) return TB_ERR_UNKNOWN_ID;
    TB_TRY(hipSetDevice(p->cfg.device));
    TB_TRY(sync_lanes(p));
    hipFree(it->second.d);
    hipFree(it->second.zap);
    p->held -= it->second.bytes + it->second.zap_bytes;
    p->series.erase(it);
    return TB_OK;
}

tb_status tb_dedisperse(tb_plan_t p, const tb_filterbank* fb, const uint8_t* data, uint32_t flags, const double* dm,
                        uint32_t ndm, float* out, uint64_t* nout, double* kernel_ms)
{
    if (!p || !fb || !data || !dm || !nout || ndm < 1 || ndm > (1u << 20) || fb->nchan < 1 || fb->nchan > 8192 ||
        fb->nsamp < 1 || fb->nsamp >= (1ull << 31) || !(fb->tsamp_s > 0.0) || !std::isfinite(fb->tsamp_s) ||
        !std::isfinite(fb->fch1_mhz) || !std::isfinite(fb->foff_mhz) || (flags != TB_MEM_HOST && flags != TB_MEM_DEVICE))
        return TB_ERR_INVALID_ARG;
    const int nbits = fb->nbits == 0 ? 8 : (int)fb->nbits;
    if (nbits != 8 && !(nbits == 4 && fb->nchan % 2 == 0)) return TB_ERR_INVALID_ARG;
    const double flast = fb->fch1_mhz + (double)(fb->nchan - 1) * fb->foff_mhz;
    if (!(std::min(fb->fch1_mhz, flast) > 0.0)) return TB_ERR_INVALID_ARG;
    for (uint32_t d = 0; d < ndm; ++d)
        if (!(dm[d] >= 0.0) || !std::isfinite(dm[d])) return TB_ERR_INVALID_ARG;
    const int nchan = (int)fb->nchan;
    const int64_t nsamp = (int64_t)fb->nsamp;
    std::vector<int32_t> delay;
    int ldd = 0;
    const int64_t smax = dedisp_delays(nchan, fb->fch1_mhz, fb->foff_mhz, fb->tsamp_s, dm, (int)ndm, delay, ldd);
    if (smax >= nsamp) return TB_ERR_INVALID_ARG;
    *nout = (uint64_t)(nsamp - smax);
    if (kernel_ms) *kernel_ms = 0.0;
    if (!out) return TB_OK;
    const int tile = dedisp_tile(), ntile = ldd / tile;
    std::vector<int2> lospan((size_t)nchan * ntile);
    for (int c = 0; c < nchan; ++c)
        for (int g = 0; g < ntile; ++g) {
            int lo = delay[(size_t)c * ldd + g * tile], hi = lo;
            for (int j = 1; j < tile; ++j) {
                const int v = delay[(size_t)c * ldd + g * tile + j];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            lospan[(size_t)c * ntile + g] = make_int2(lo, hi - lo);
        }
    std::lock_guard<std::mutex> lk(p->mu);
    TB_TRY(hipSetDevice(p->cfg.device));
    // scratch: [time-major copy of host data] channel-major bytes, delays, tile bounds
    const size_t bytes = (size_t)nchan * (size_t)nsamp / (nbits == 4 ? 2 : 1);  // packed input
    const int64_t ldx = (nsamp + 15) & ~(int64_t)15;  // channel-major rows, 16-byte aligned
    const size_t bcm = (size_t)nchan * (size_t)ldx;
    const size_t bdel = sizeof(int32_t) * delay.size(), blo = sizeof(int2) * lospan.size();
    uint8_t *d_tm = nullptr, *d_cm = nullptr;
    int32_t* d_delay = nullptr;
    int2* d_lospan = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    tb_status st = TB_OK;
    if ((flags == TB_MEM_HOST && hipMalloc(&d_tm, bytes) != hipSuccess) || hipMalloc(&d_cm, bcm) != hipSuccess ||
        hipMalloc(&d_delay, bdel) != hipSuccess || hipMalloc(&d_lospan, blo) != hipSuccess)
        st = TB_ERR_OOM;
    const uint8_t* src = flags == TB_MEM_HOST ? d_tm : data;
    if (!st && ((flags == TB_MEM_HOST && hipMemcpyAsync(d_tm, data, bytes, hipMemcpyHostToDevice, p->stream) != hipSuccess) ||
                hipMemcpyAsync(d_delay, delay.data(), bdel, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
                hipMemcpyAsync(d_lospan, lospan.data(), blo, hipMemcpyHostToDevice, p->stream) != hipSuccess))
        st = TB_ERR_DEVICE;
    if (!st && kernel_ms && (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess ||
                             hipEventRecord(ev[0], p->stream) != hipSuccess))
        st = TB_ERR_DEVICE;
    if (!st && launch_dedisperse(src, nbits, d_cm, nchan, nsamp, ldx, d_delay, ldd, d_lospan, (int)ndm,
                                 (int64_t)*nout, out, p->stream) != hipSuccess)
        st = TB_ERR_DEVICE;
    if (!st && kernel_ms && hipEventRecord(ev[1], p->stream) != hipSuccess) st = TB_ERR_DEVICE;
    if (hipStreamSynchronize(p->stream) != hipSuccess && !st) st = TB_ERR_DEVICE;
    if (!st && kernel_ms) {
        float f = 0.0f;
        if (hipEventElapsedTime(&f, ev[0], ev[1]) != hipSuccess) st = TB_ERR_DEVICE;
        *kernel_ms = f;
    }
    for (hipEvent_t e : ev)
        if (e) hipEventDestroy(e);
    hipFree(d_tm);
    hipFree(d_cm);
    hipFree(d_delay);
    hipFree(d_lospan);
    return st;
}

tb_status tb_bank_density(tb_plan_t p, const tb_bank_metric* m, const tb_template* pts, uint64_t count,
                          double* out, double* kernel_ms)
{
    if (!p || !m || (count && (!pts || !out)) || count > (1ull << 31) || (m->kind != TB_BANK_CIRCULAR &&
        m->kind != TB_BANK_ELLIPTICAL) || m->nodes < 8 || m->nodes > 8192 || !(m->tobs_s > 0.0) ||
        !std::isfinite(m->tobs_s) || !(m->fmax_hz > 0.0) || !std::isfinite(m->fmax_hz))
        return TB_ERR_INVALID_ARG;
    for (uint64_t i = 0; i < count; ++i) {
        const tb_template& t = pts[i];
        if (!valid_template(t)) return TB_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(p->mu);
    TB_TRY(hipSetDevice(p->cfg.device));
    if (kernel_ms) *kernel_ms = 0.0;
    if (count == 0) return TB_OK;
    tb_template* d_pts = nullptr;
    double* d_out = nullptr;
    const size_t bp = sizeof(tb_template) * count, bo = sizeof(double) * count;
    tb_status st = TB_OK;
    if (hipMalloc(&d_pts, bp) != hipSuccess || hipMalloc(&d_out, bo) != hipSuccess) st = TB_ERR_OOM;
    if (!st && (hipMemcpyAsync(d_pts, pts, bp, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
                launch_bank_density((int)m->kind, (int)m->nodes, m->tobs_s, m->fmax_hz, d_pts, (uint32_t)count, d_out,
                                    p->stream, kernel_ms) != hipSuccess ||
                hipMemcpy(out, d_out, bo, hipMemcpyDeviceToHost) != hipSuccess))
        st = TB_ERR_DEVICE;
    hipStreamSynchronize(p->stream);
    hipFree(d_pts);
    hipFree(d_out);
    return st;
}

tb_status tb_bank_propose(tb_plan_t p, const tb_bank_metric* m, const tb_bank_priors* pr, const double* u,
                          uint64_t count, tb_template* points, double* weights, double* stats, double* kernel_ms)
{
    if (!p || !m || !pr || (count && !u) || (stats && count < 2) || count > (1ull << 31)) return TB_ERR_INVALID_ARG;
    const bool ell = m->kind == TB_BANK_ELLIPTICAL;
    if (!(pr->porb_min_s > 0.0) || !(pr->porb_max_s >= pr->porb_min_s) || !std::isfinite(pr->porb_max_s) ||
        !(pr->m_pulsar_min_msun > 0.0) || !(pr->m_comp_max_msun > 0.0) || !std::isfinite(pr->m_pulsar_min_msun) ||
        !std::isfinite(pr->m_comp_max_msun) || (ell && !(pr->ecc_max > 0.0 && pr->ecc_max < 1.0)))
        return TB_ERR_INVALID_ARG;
    const int d = ell ? 5 : 3;
    for (uint64_t i = 0; i < count * (uint64_t)d; ++i)
        if (!(u[i] >= 0.0 && u[i] < 1.0)) return TB_ERR_INVALID_ARG;
    // G M_sun / c^3 [s]
    const double tsun = 4.925490947e-6;
    const double span = pr->porb_max_s - pr->porb_min_s;
    std::vector<tb_template> pts((size_t)count);
    std::vector<double> pdf((size_t)count), dens((size_t)count);
    for (uint64_t i = 0; i < count; ++i) {
        const double* ui = u + (size_t)i * d;
        tb_template& t = pts[(size_t)i];
        t.porb_s = pr->porb_min_s + span * ui[0];
        const double om = 2.0 * kPi / t.porb_s;
        const double tau_max = std::cbrt(tsun) * std::pow(om, -2.0 / 3.0) * pr->m_comp_max_msun /
                               std::pow(pr->m_pulsar_min_msun + pr->m_comp_max_msun, 2.0 / 3.0);
        t.tau_lts = ui[1] * tau_max;
        t.alpha_rad = 2.0 * kPi * ui[2];
        double q = 1.0 / ((span > 0.0 ? span : 1.0) * tau_max * 2.0 * kPi);
        t.ecc = 0.0;
        t.omega_rad = 0.0;
        if (ell) {
            t.ecc = pr->ecc_max * ui[3];
            t.omega_rad = 2.0 * kPi * ui[4];
            q /= pr->ecc_max * 2.0 * kPi;
        }
        pdf[(size_t)i] = q;
    }
    tb_status st = tb_bank_density(p, m, pts.data(), count, dens.data(), kernel_ms);
    if (st) return st;
    double sw = 0.0, sw2 = 0.0, wmax = 0.0;
    for (uint64_t i = 0; i < count; ++i) {
        const double w = dens[(size_t)i] / pdf[(size_t)i];
        if (weights) weights[i] = w;
        sw += w;
        sw2 += w * w;
        wmax = std::max(wmax, w);
    }
    if (points) std::memcpy(points, pts.data(), sizeof(tb_template) * (size_t)count);
    if (stats) {
        const double n = (double)count, mean = sw / n;
        const double var = std::max(0.0, (sw2 - n * mean * mean) / (n - 1.0));
        stats[0] = mean;
        stats[1] = std::sqrt(var / n);
        stats[2] = wmax;
    }
    return TB_OK;
}

tb_status tb_bank_count(double volume, uint32_t n, double coverage, double mismatch, double* count)
{
    if (!count || !(volume > 0.0) || !std::isfinite(volume) || !(coverage > 0.0 && coverage < 1.0) ||
        !(mismatch > 0.0) || !std::isfinite(mismatch) || n < 1 || n > 16)
        return TB_ERR_INVALID_ARG;
    const double h = 0.5 * (double)n;
    const double cn = std::pow(kPi, h) / std::tgamma(h + 1.0);
    const double x = std::pow(mismatch, h) * cn / volume;
    if (!(x < 1.0)) return TB_ERR_INVALID_ARG;
    *count = std::log(1.0 - coverage) / std::log1p(-x);
    return TB_OK;
}

tb_status tb_bank_select(const double* weights, const double* u, uint64_t count, double wmax, uint8_t* keep,
                         uint64_t* n_keep, uint64_t* n_above)
{
    if ((count && (!weights || !u || !keep)) || !(wmax > 0.0) || !std::isfinite(wmax)) return TB_ERR_INVALID_ARG;
    uint64_t k = 0, a = 0;
    for (uint64_t i = 0; i < count; ++i) {
        keep[i] = (uint8_t)(u[i] * wmax < weights[i]);
        k += keep[i];
        a += weights[i] > wmax;
    }
    if (n_keep) *n_keep = k;
    if (n_above) *n_above = a;
    return TB_OK;
}

tb_status tb_set_shape(tb_plan_t p, uint32_t log2n, uint32_t tile_points, uint32_t batch_templates)
{
    if (!p || log2n < 10 || log2n > p->cfg.max_log2n ||
        (tile_points != 0 && tile_points != 8192 && tile_points != 16384) || batch_templates > 4096)
        return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->geo.count((int)log2n)) return TB_ERR_INVALID_ARG;  // that length is already laid out
    for (const auto& L : p->lanes)
        if (L.slots.count((int)log2n)) return TB_ERR_INVALID_ARG;
    p->shape[(int)log2n] = std::make_pair((int)tile_points, (int)batch_templates);
    return TB_OK;
}

tb_status tb_zap_series(tb_plan_t p, int32_t sid, const double* lo_hz, const double* hi_hz, uint32_t count)
{
    if (!p || (count && (!lo_hz || !hi_hz)) || count > TB_ZAP_MAX) return TB_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < count; ++i)
        if (!std::isfinite(lo_hz[i]) || !std::isfinite(hi_hz[i])) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->series.find(sid);
    if (it == p->series.end()) return TB_ERR_UNKNOWN_ID;
    SeriesRec& sr = it->second;
    // bins k with lo <= k / T <= hi, 1 <= k <= M; merged into disjoint ranges
    const double T = (double)sr.n * sr.tsamp;
    const int64_t M = sr.n / 2;
    std::vector<std::pair<int64_t, int64_t>> r;
    for (uint32_t i = 0; i < count; ++i) {
        const double lo = std::ceil(lo_hz[i] * T), hi = std::floor(hi_hz[i] * T);
        const int64_t a = lo < 1.0 ? 1 : (lo > (double)M ? M + 1 : (int64_t)lo);
        const int64_t b = hi > (double)M ? M : (hi < 0.0 ? 0 : (int64_t)hi);
        if (a <= b) r.emplace_back(a, b);
    }
    std::sort(r.begin(), r.end());
    std::vector<int2> merged;
    for (const auto& ab : r) {
        if (!merged.empty() && ab.first <= (int64_t)merged.back().y + 1)
            merged.back().y = (int)std::max<int64_t>(merged.back().y, ab.second);
        else
            merged.push_back(make_int2((int)ab.first, (int)ab.second));
    }
    TB_TRY(hipSetDevice(p->cfg.device));
    TB_TRY(sync_lanes(p));
    Geometry* g = nullptr;
    tb_status st = get_geometry(p, ilog2((uint64_t)sr.n), &g);
    if (st) return st;
    int2* dz = nullptr;
    const size_t bytes = sizeof(int2) * merged.size();
    if (bytes) {
        if ((st = reserve(p, bytes))) return st;
        if (hipMalloc(&dz, bytes) != hipSuccess) {
            p->held -= bytes;
            return TB_ERR_OOM;
        }
        if (hipMemcpy(dz, merged.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            hipFree(dz);
            p->held -= bytes;
            return TB_ERR_DEVICE;
        }
    }
    hipFree(sr.zap);
    p->held -= sr.zap_bytes;
    sr.zap = dz;
    sr.nzap = (int)merged.size();
    sr.zap_bytes = bytes;
    // a series whitened once carries the ranges in its factors
    if (sr.fac && (launch_series_factors(*g, sr.med, sr.fac, sr.zap, sr.nzap, p->stream) != hipSuccess ||
                   hipStreamSynchronize(p->stream) != hipSuccess))
        return TB_ERR_DEVICE;
    return TB_OK;
}

tb_status tb_search_templates(tb_plan_t p, int32_t sid, const tb_template* t, uint32_t count, uint32_t first,
                              int64_t* request_id)
{
    if (!p || !request_id || (count && !t)) return TB_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < count; ++i)
        if (!valid_template(t[i])) return TB_ERR_INVALID_ARG;
    if ((uint64_t)first + count > 0xffffffffull) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto sit = p->series.find(sid);
    if (sit == p->series.end()) return TB_ERR_UNKNOWN_ID;
    TB_TRY(hipSetDevice(p->cfg.device));
    const SeriesRec& sr = sit->second;
    for (uint32_t i = 0; i < count; ++i)
        if (!delay_fits(p, t[i], sr.tsamp)) return TB_ERR_INVALID_ARG;
    Geometry* g = nullptr;
    Slots* ws = nullptr;
    tb_status st;
    if ((st = get_geometry(p, ilog2((uint64_t)sr.n), &g))) return st;
    int lane = pick_lane(p);
    if ((st = get_slots(p, lane, *g, &ws))) {
        // no room for another workspace: queue behind a lane that has one
        int other = -1;
        for (int l = 0; l < (int)p->lanes.size(); ++l)
            if (p->lanes[l].slots.count(g->log2n) && (other < 0 || p->lanes[l].pending < p->lanes[other].pending))
                other = l;
        if (st != TB_ERR_BUDGET || other < 0) return st;
        lane = other;
        if ((st = get_slots(p, lane, *g, &ws))) return st;
    }
    hipStream_t stream = p->lanes[lane].stream;

    Req r;
    r.lane = lane;
    r.work = (double)count * (double)sr.n;
    r.series = sid;
    r.count = count;
    r.first = first;
    r.cap = p->cfg.ring_capacity;
    r.n = sr.n;
    r.tsamp = sr.tsamp;
    ReqLayout L = req_layout(count, r.cap);
    r.bytes = L.total;
    if ((st = reserve(p, r.bytes))) return st;
    if (!(r.dmem = take_device(p, L.total, &r.dmem_size))) {
        p->held -= r.bytes;
        return TB_ERR_OOM;
    }
    if (count && !(r.h_t = take_pinned(p, sizeof(tb_template) * count, &r.h_t_size))) {
        free_request(p, r);
        p->held -= r.bytes;
        return TB_ERR_OOM;
    }
    if (count) std::memcpy(r.h_t, t, sizeof(tb_template) * count);
    tb_template* d_t = (tb_template*)(r.dmem + L.off_t);
    TmplDev* d_tm = (TmplDev*)(r.dmem + L.off_tm);
    uint32_t* counter = (uint32_t*)(r.dmem + L.off_cnt);
    uint4* ring = (uint4*)(r.dmem + L.off_ring);
    PeakParams pp = peak_params(p, sr.n, sr.tsamp, (uint32_t)sid, first, r.cap);
    if (hipEventCreate(&r.ev0) != hipSuccess || hipEventCreate(&r.ev1) != hipSuccess ||
        hipEventRecord(r.ev0, stream) != hipSuccess || launch_fill_u32(counter, 0u, 1, stream) != hipSuccess ||
        (count && hipMemcpyAsync(d_t, r.h_t, sizeof(tb_template) * count, hipMemcpyHostToDevice, stream) !=
                      hipSuccess) ||
        launch_template_prep(d_t, count, d_tm, delay_model(p), stream) != hipSuccess) {
        hipStreamSynchronize(stream);
        free_request(p, r);
        p->held -= r.bytes;
        return TB_ERR_DEVICE;
    }
    // Idle lanes (no queued work) help with requests of more than one wave:
    // they wait for the prepared templates, take every k-th wave on their own
    // workspace, and the primary lane waits for them before the completion
    // event.  All waves append to the request's one candidate ring.
    Crew crew;
    crew.streams.push_back(stream);
    crew.slots.push_back(ws);
    if (count > (uint32_t)ws->B) {
        for (int l = 0; l < (int)p->lanes.size() && crew.streams.size() * (size_t)ws->B < count; ++l) {
            Slots* hs = nullptr;
            if (l == lane || p->lanes[l].pending > 0.0 || get_slots(p, l, *g, &hs) != TB_OK) continue;
            crew.streams.push_back(p->lanes[l].stream);
            crew.slots.push_back(hs);
            r.parts.emplace_back(l, 0.0);
        }
    }
    auto fail = [&](tb_status why) {
        for (hipStream_t cs : crew.streams) hipStreamSynchronize(cs);
        free_request(p, r);
        p->held -= r.bytes;
        return why;
    };
    if (crew.streams.size() > 1) {
        hipEvent_t ready = nullptr;
        if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return fail(TB_ERR_DEVICE);
        r.joins.push_back(ready);
        if (hipEventRecord(ready, stream) != hipSuccess) return fail(TB_ERR_DEVICE);
        for (size_t c = 1; c < crew.streams.size(); ++c)
            if (hipStreamWaitEvent(crew.streams[c], ready, 0) != hipSuccess) return fail(TB_ERR_DEVICE);
    }
    Inspect none;
    st = enqueue(p, crew, sr, g, d_tm, count, pp, ring, counter, none);
    if (st) return fail(st);
    for (size_t c = 1; c < crew.streams.size(); ++c) {
        hipEvent_t done = nullptr;
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) return fail(TB_ERR_DEVICE);
        r.joins.push_back(done);
        if (hipEventRecord(done, crew.streams[c]) != hipSuccess || hipStreamWaitEvent(stream, done, 0) != hipSuccess)
            return fail(TB_ERR_DEVICE);
    }
    if (launch_significance(ring, counter, r.cap, stream) != hipSuccess || hipEventRecord(r.ev1, stream) != hipSuccess)
        return fail(TB_ERR_DEVICE);
    // pending work split by waves taken
    {
        const size_t nc = crew.streams.size(), nw = (count + (uint32_t)ws->B - 1) / (uint32_t)ws->B;
        const double per_wave = nw ? r.work / (double)nw : 0.0;
        std::vector<double> share(nc, 0.0);
        for (size_t i = 0; i < nw; ++i) share[i % nc] += per_wave;
        r.parts.insert(r.parts.begin(), std::make_pair(lane, 0.0));
        for (size_t c = 0; c < nc; ++c) {
            r.parts[c].second = share[c];
            p->lanes[r.parts[c].first].pending += share[c];
        }
    }
    int64_t rid = p->next_req++;
    p->reqs.emplace(rid, std::move(r));
    *request_id = rid;
    return TB_OK;
}

tb_status tb_search_templates_noalloc(tb_plan_t p, int32_t sid, const tb_template* t, uint32_t count,
                                      uint32_t first, tb_candidate* out, uint64_t capacity, uint64_t* n_total)
{
    if (!p || !n_total || (count && !t) || (capacity && !out) || capacity > 0xffffffffull)
        return TB_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < count; ++i)
        if (!valid_template(t[i])) return TB_ERR_INVALID_ARG;
    if ((uint64_t)first + count > 0xffffffffull) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto sit = p->series.find(sid);
    if (sit == p->series.end()) return TB_ERR_UNKNOWN_ID;
    TB_TRY(hipSetDevice(p->cfg.device));
    const SeriesRec& sr = sit->second;
    for (uint32_t i = 0; i < count; ++i)
        if (!delay_fits(p, t[i], sr.tsamp)) return TB_ERR_INVALID_ARG;
    // the series' length was laid out (tables, tile order) when it was loaded
    auto git = p->geo.find(ilog2((uint64_t)sr.n));
    char* base = scratch_of(p->cfg.device);
    if (git == p->geo.end() || !base) return TB_ERR_DEVICE;
    const Geometry& g = git->second.g;
    ScratchLayout L;
    if (!scratch_layout(p, g, count, capacity, &L)) return TB_ERR_TOO_LARGE;
    Slots ws = L.ws;
    ws.Y = (float2*)(base + L.off_y);
    ws.P = (float*)(base + L.off_p);
    ws.Q = (float*)(base + L.off_w);
    ws.med = (float*)(base + L.off_m);
    ws.poly = (ChunkPoly*)(base + L.off_q);
    ws.pok = (int32_t*)(base + L.off_k);
    tb_template* d_t = (tb_template*)(base + L.req.off_t);
    TmplDev* d_tm = (TmplDev*)(base + L.req.off_tm);
    uint32_t* counter = (uint32_t*)(base + L.req.off_cnt);
    uint4* ring = (uint4*)(base + L.req.off_ring);
    hipStream_t s = p->stream;
    const PeakParams pp = peak_params(p, sr.n, sr.tsamp, (uint32_t)sid, first, capacity);
    // the counter starts at zero (a fill kernel, not a memset)
    hipError_t e = launch_fill_u32(counter, 0u, 1, s);
    if (e == hipSuccess && count)
        e = hipMemcpyAsync(d_t, t, sizeof(tb_template) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_template_prep(d_t, count, d_tm, delay_model(p), s);
    const Inspect none;
    for (uint32_t w0 = 0; w0 < count && e == hipSuccess;) {
        const int nslots = (int)std::min<uint32_t>((uint32_t)ws.B, count - w0);
        e = launch_wave(g, sr.d, sr.tsamp, d_tm, (int)w0, nslots, ws, sr.fac, sr.zap, sr.nzap, pp, ring, counter,
                        none, s, nullptr);
        w0 += (uint32_t)nslots;
    }
    if (e == hipSuccess) e = launch_significance(ring, counter, capacity, s);
    uint32_t total = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&total, counter, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const uint64_t keep = std::min<uint64_t>(total, capacity);
    if (e == hipSuccess && keep) e = hipMemcpyAsync(out, ring, keep * sizeof(uint4), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return TB_ERR_DEVICE;
    // The 16-byte ring records now fill the front of out; widen them in place
    // from the last one down.  Candidate i covers the bytes of records 2i and
    // 2i + 1, which are read (i = 0) or already widened (i > 0) by then.
    static_assert(sizeof(tb_candidate) == 2 * sizeof(uint4), "candidate record sizes");
    const double T = (double)sr.n * sr.tsamp;
    for (uint64_t i = keep; i-- > 0;) {
        uint4 q;
        std::memcpy(&q, (const char*)out + i * sizeof(uint4), sizeof(q));
        tb_candidate c;
        to_candidate(q, (uint32_t)sid, T, c);
        std::memcpy(&out[i], &c, sizeof(c));
    }
    sort_candidates(out, (size_t)keep);
    *n_total = total;
    return total > capacity ? TB_ERR_OVERFLOW : TB_OK;
}

tb_status tb_poll(tb_plan_t p, int64_t rid)
{
    if (!p) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->reqs.find(rid);
    if (it == p->reqs.end()) return TB_ERR_UNKNOWN_ID;
    hipError_t e = hipEventQuery(it->second.ev1);
    if (e == hipSuccess) return TB_OK;
    if (e == hipErrorNotReady) return TB_ERR_NOT_READY;
    return TB_ERR_DEVICE;
}

tb_status tb_get_candidates(tb_plan_t p, int64_t rid, tb_candidate* out, uint64_t capacity, uint64_t* n_total,
                            int blocking)
{
    if (!p || !n_total) return TB_ERR_INVALID_ARG;
    hipEvent_t ev;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        auto it = p->reqs.find(rid);
        if (it == p->reqs.end()) return TB_ERR_UNKNOWN_ID;
        ev = it->second.ev1;
        if (!it->second.fetched) {
            hipError_t e = hipEventQuery(ev);
            if (e == hipErrorNotReady && !blocking) return TB_ERR_NOT_READY;
            if (e != hipSuccess && e != hipErrorNotReady) return TB_ERR_DEVICE;
        }
    }
    TB_TRY(hipSetDevice(p->cfg.device));
    TB_TRY(hipEventSynchronize(ev));
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->reqs.find(rid);
    if (it == p->reqs.end()) return TB_ERR_UNKNOWN_ID;
    Req& r = it->second;
    tb_status st = fetch(p, r);
    if (st) return st;
    *n_total = r.total;
    if (out) {
        size_t k = (size_t)std::min<uint64_t>(capacity, r.cands.size());
        if (k) std::memcpy(out, r.cands.data(), k * sizeof(tb_candidate));
    }
    return r.total > r.cap ? TB_ERR_OVERFLOW : TB_OK;
}

tb_status tb_release(tb_plan_t p, int64_t rid)
{
    if (!p) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->reqs.find(rid);
    if (it == p->reqs.end()) return TB_ERR_UNKNOWN_ID;
    TB_TRY(hipSetDevice(p->cfg.device));
    TB_TRY(hipEventSynchronize(it->second.ev1));
    if (!it->second.settled)
        for (auto& pw : it->second.parts) p->lanes[pw.first].pending -= pw.second;
    p->held -= it->second.bytes;
    free_request(p, it->second);
    p->reqs.erase(it);
    return TB_OK;
}

tb_status tb_synchronize(tb_plan_t p)
{
    if (!p) return TB_ERR_INVALID_ARG;
    TB_TRY(hipSetDevice(p->cfg.device));
    TB_TRY(sync_lanes(p));
    return TB_OK;
}

tb_status tb_memory(tb_plan_t p, uint64_t* held, uint64_t* budget)
{
    if (!p) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    if (held) *held = p->held;
    if (budget) *budget = p->cfg.hbm_budget_bytes;
    return TB_OK;
}

tb_status tb_set_budget(tb_plan_t p, uint64_t budget)
{
    if (!p) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    p->cfg.hbm_budget_bytes = budget;
    return TB_OK;
}

tb_status tb_thresholds(tb_plan_t p, float out[5])
{
    if (!p || !out) return TB_ERR_INVALID_ARG;
    for (int l = 0; l < 5; ++l) out[l] = (float)p->thr[l];
    return TB_OK;
}

tb_status tb_last_request_ms(tb_plan_t p, int64_t rid, double* ms)
{
    if (!p || !ms) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->reqs.find(rid);
    if (it == p->reqs.end()) return TB_ERR_UNKNOWN_ID;
    TB_TRY(hipEventSynchronize(it->second.ev1));
    float f = 0.0f;
    TB_TRY(hipEventElapsedTime(&f, it->second.ev0, it->second.ev1));
    *ms = f;
    return TB_OK;
}

tb_status tb_profile(tb_plan_t p, int every)
{
    if (!p || every < 0) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    if (every) {
        TB_TRY(hipSetDevice(p->cfg.device));
        TB_TRY(sync_lanes(p));
        for (auto& v : p->prof_events)
            for (auto& m : v) hipEventDestroy(m.second);
        p->prof_events.clear();
        p->prof_templates = 0;
        p->prof_wave = 0;
    }
    p->prof_every = (uint32_t)every;
    return TB_OK;
}

tb_status tb_profile_read(tb_plan_t p, double ms[6], uint64_t launches[6], uint64_t* templates)
{
    if (!p) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    TB_TRY(hipSetDevice(p->cfg.device));
    TB_TRY(sync_lanes(p));
    double acc[K_CLASSES] = {0, 0, 0, 0, 0, 0};
    uint64_t cnt[K_CLASSES] = {0, 0, 0, 0, 0, 0};
    for (auto& v : p->prof_events)
        for (size_t i = 0; i + 1 < v.size(); ++i) {
            const int k = v[i].first;
            if (k < 0 || k >= K_CLASSES) continue;
            float f = 0.0f;
            TB_TRY(hipEventElapsedTime(&f, v[i].second, v[i + 1].second));
            acc[k] += f;
            cnt[k] += 1;
        }
    for (int k = 0; k < K_CLASSES; ++k) {
        if (ms) ms[k] = acc[k];
        if (launches) launches[k] = cnt[k];
    }
    if (templates) *templates = p->prof_templates;
    return TB_OK;
}

tb_status tb_stream_copy(tb_plan_t p, void* dst, const void* src, uint64_t bytes, uint32_t reps, double* ms)
{
    if (!p || !dst || !src || !ms || bytes == 0 || (bytes & 15) || reps == 0) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    TB_TRY(hipSetDevice(p->cfg.device));
    hipEvent_t a = nullptr, b = nullptr;
    TB_TRY(hipEventCreate(&a));
    TB_TRY(hipEventCreate(&b));
    hipError_t e = launch_copy((float4*)dst, (const float4*)src, bytes / 16, p->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, p->stream);
    for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy((float4*)dst, (const float4*)src, bytes / 16, p->stream);
    if (e == hipSuccess) e = hipEventRecord(b, p->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float f = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (e != hipSuccess) return TB_ERR_DEVICE;
    *ms = (double)f / reps;
    return TB_OK;
}

tb_status tb_inspect_template(tb_plan_t p, int32_t sid, const tb_template* t, int32_t* src, float* power,
                              float* medians, float* sums)
{
    if (!p || !t || !valid_template(*t)) return TB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    auto sit = p->series.find(sid);
    if (sit == p->series.end()) return TB_ERR_UNKNOWN_ID;
    TB_TRY(hipSetDevice(p->cfg.device));
    const SeriesRec& sr = sit->second;
    if (!delay_fits(p, *t, sr.tsamp)) return TB_ERR_INVALID_ARG;
    Geometry* g = nullptr;
    Slots* ws = nullptr;
    tb_status st;
    if ((st = get_geometry(p, ilog2((uint64_t)sr.n), &g))) return st;
    if ((st = get_slots(p, 0, *g, &ws))) return st;
    int nfold = ilog2(p->cfg.harm_max) + 1;
    size_t nb = (size_t)g->M + 1;
    // [0, 256) prepared template, [256, 320) template, [512, 768) counter,
    // [768, 1024) ring, then indices, fold sums, power
    static_assert(sizeof(TmplDev) <= 256, "inspection layout");
    const size_t off_src = 1024;
    size_t need = off_src + sizeof(int32_t) * (size_t)sr.n + sizeof(float) * nfold * nb + sizeof(float) * nb;
    char* d = nullptr;
    tb_template* ht = nullptr;
    if (hipMalloc(&d, need) != hipSuccess) return TB_ERR_OOM;
    if (hipHostMalloc(&ht, sizeof(tb_template), hipHostMallocDefault) != hipSuccess) {
        hipFree(d);
        return TB_ERR_OOM;
    }
    *ht = *t;
    TmplDev* d_tm = (TmplDev*)d;
    tb_template* d_t = (tb_template*)(d + 256);
    uint32_t* counter = (uint32_t*)(d + 512);
    uint4* ring = (uint4*)(d + 768);
    Inspect ins;
    ins.src = (int32_t*)(d + off_src);
    ins.sums = (float*)((char*)ins.src + sizeof(int32_t) * (size_t)sr.n);
    ins.power = ins.sums + (size_t)nfold * nb;
    float* const d_power = ins.power;
    PeakParams pp = peak_params(p, sr.n, sr.tsamp, (uint32_t)sid, 0, 0);
    st = TB_OK;
    if (launch_fill_u32(counter, 0u, 1, p->stream) != hipSuccess ||
        hipMemcpyAsync(d_t, ht, sizeof(tb_template), hipMemcpyHostToDevice, p->stream) != hipSuccess ||
        launch_template_prep(d_t, 1, d_tm, delay_model(p), p->stream) != hipSuccess)
        st = TB_ERR_DEVICE;
    if (!st && sr.fac && power) {
        // a series whitened once: pass 2 of the search stores whitened power,
        // so the raw power comes from a pass without the factors
        Inspect raw;
        raw.power = ins.power;
        if (launch_wave(*g, sr.d, sr.tsamp, d_tm, 0, 1, *ws, nullptr, nullptr, 0, pp, ring, counter, raw,
                        p->stream) !=
            hipSuccess)
            st = TB_ERR_DEVICE;
        ins.power = nullptr;
    }
    Crew crew;
    crew.streams.push_back(p->stream);
    crew.slots.push_back(ws);
    if (!st) st = enqueue(p, crew, sr, g, d_tm, 1, pp, ring, counter, ins);
    if (!st && hipStreamSynchronize(p->stream) != hipSuccess) st = TB_ERR_DEVICE;
    if (!st && src && hipMemcpy(src, ins.src, sizeof(int32_t) * (size_t)sr.n, hipMemcpyDeviceToHost) != hipSuccess)
        st = TB_ERR_DEVICE;
    if (!st && power &&
        hipMemcpy(power, d_power, sizeof(float) * nb, hipMemcpyDeviceToHost) != hipSuccess)
        st = TB_ERR_DEVICE;
    if (!st && medians &&
        hipMemcpy(medians, sr.fac ? sr.med : ws->med, sizeof(float) * (size_t)g->nblk, hipMemcpyDeviceToHost) !=
            hipSuccess)
        st = TB_ERR_DEVICE;
    if (!st && sums && hipMemcpy(sums, ins.sums, sizeof(float) * nfold * nb, hipMemcpyDeviceToHost) != hipSuccess)
        st = TB_ERR_DEVICE;
    hipStreamSynchronize(p->stream);
    hipFree(d);
    hipHostFree(ht);
    return st;
}

}  // extern "C"

uint64_t tb::plan_ring_capacity(tb_plan_t p) { return p ? p->cfg.ring_capacity : 0; }
