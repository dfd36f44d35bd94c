// runtime.hip -- host runtime behind the C ABI of include/sevo.h: contexts,
// error plumbing, the instance generator and cache, descriptor staging and
// the dispatch of evaluation batches to the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sevo.h"
#include "runtime.h"
#include "state.h"

using namespace sevo;

// ---------------------------------------------------------------------------
// Instances

namespace sevo {

// Orthogonal factor of a Householder QR of the n x n row-major matrix G with
// every diagonal entry of R made positive (so the factor is unique).  The
// reflectors are stored column by column and accumulated backwards onto the
// identity.
static void orthogonal_factor(int n, std::vector<double> G, std::vector<double> &Q)
{
    std::vector<std::vector<double>> refl;   // refl[k][r - k], unit norm
    std::vector<int> flip(n, 0);
    refl.reserve(n);
    auto at = [&](int r, int c) -> double & { return G[(size_t)r * n + c]; };
    for (int k = 0; k < n; ++k) {
        std::vector<double> v(n - k);
        double nrm = 0.0;
        for (int r = k; r < n; ++r) { v[r - k] = at(r, k); nrm += v[r - k] * v[r - k]; }
        nrm = std::sqrt(nrm);
        if (k == n - 1 || nrm == 0.0) {
            // last column (or a zero one): no reflector; R_kk = at(k, k)
            refl.emplace_back();
            flip[k] = at(k, k) < 0.0;
            continue;
        }
        const double alpha = v[0] >= 0.0 ? -nrm : nrm;   // R_kk after the reflection
        v[0] -= alpha;
        double vn = 0.0;
        for (double e : v) vn += e * e;
        vn = std::sqrt(vn);
        if (vn == 0.0) { refl.emplace_back(); flip[k] = at(k, k) < 0.0; continue; }
        for (double &e : v) e /= vn;
        for (int c = k; c < n; ++c) {
            double dot = 0.0;
            for (int r = k; r < n; ++r) dot += v[r - k] * at(r, c);
            for (int r = k; r < n; ++r) at(r, c) -= 2.0 * dot * v[r - k];
        }
        flip[k] = alpha < 0.0;
        refl.push_back(std::move(v));
    }
    // Q = H_0 H_1 ... H_{n-1} I, applied right to left.
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int k = n - 1; k >= 0; --k) {
        const std::vector<double> &v = refl[k];
        if (v.empty()) continue;
        for (int c = 0; c < n; ++c) {
            double dot = 0.0;
            for (int r = k; r < n; ++r) dot += v[r - k] * Q[(size_t)r * n + c];
            for (int r = k; r < n; ++r) Q[(size_t)r * n + c] -= 2.0 * dot * v[r - k];
        }
    }
    for (int j = 0; j < n; ++j)
        if (flip[j])
            for (int r = 0; r < n; ++r) Q[(size_t)r * n + j] = -Q[(size_t)r * n + j];
}

static void generate_instance(int func, int dim, uint32_t inst, uint64_t inst_seed,
                              std::vector<double> &o, std::vector<double> &M)
{
    const uint32_t k1 = fold_seed(inst_seed);
    o.assign(dim, 0.0);
    for (int j = 0; j < dim; j += 2) {
        const u32x4 w = draw(inst, k1, (uint32_t)func, (uint32_t)dim, TAG_SHIFT_O, (uint32_t)(j >> 1));
        o[j] = -80.0 + 160.0 * u53(w.x, w.y);
        if (j + 1 < dim) o[j + 1] = -80.0 + 160.0 * u53(w.z, w.w);
    }
    const size_t nn = (size_t)dim * dim;
    std::vector<double> G(nn);
    const double two_pi = 6.283185307179586476925287;
    for (size_t e = 0; e < nn; e += 2) {
        const u32x4 w = draw(inst, k1, (uint32_t)func, (uint32_t)dim, TAG_ROT_N, (uint32_t)(e >> 1));
        const double rad = std::sqrt(-2.0 * std::log(1.0 - u53(w.x, w.y)));
        const double ang = two_pi * u53(w.z, w.w);
        G[e] = rad * std::cos(ang);
        if (e + 1 < nn) G[e + 1] = rad * std::sin(ang);
    }
    orthogonal_factor(dim, std::move(G), M);
}

Consts make_consts()
{
    Consts k;
    const double s = SCHWEFEL_S, a = std::sqrt(s);
    const double c = s * std::sin(a);
    const double s500 = std::sin(std::sqrt(500.0));
    SchwefelConst<double> d;
    d.s = s; d.a = a; d.sa = std::sin(a); d.ca = std::cos(a); d.c = c;
    d.zhi = 500.0 - s; d.zlo = -500.0 - s;
    d.gp = c - 500.0 * s500; d.gm = c + 500.0 * s500;
    d.lambda = SCHWEFEL_LAMBDA; d.nega_s = -s;
    k.kd = d;
    k.kf = SchwefelConst<float>{(float)d.s, (float)d.a, (float)d.sa, (float)d.ca, (float)d.c,
                                (float)d.zhi, (float)d.zlo, (float)d.gp, (float)d.gm,
                                (float)d.lambda, (float)d.nega_s};
    return k;
}

}  // namespace sevo

// ---------------------------------------------------------------------------
// Context

struct DevInstance {
    int func = 0, dim = 0;
    std::vector<double> o, M;
    double *d_o = nullptr, *d_M64 = nullptr;
    float *d_Mfrag = nullptr, *d_tab = nullptr;
    uint16_t *d_Mbf = nullptr;
};

struct DescSlot {
    char *h = nullptr, *d = nullptr;
    size_t cap = 0, used = 0;
    bool valid = false;          // device copy equals h[0, used)
    hipEvent_t done = nullptr;   // recorded after the latest reader's kernels
    hipStream_t stream = nullptr;   // the stream of the latest reader
};

// The device array behind sevo_evaluate_batch_noalloc: the descriptor tables
// of one call, packed at 256-byte offsets.  Every GPU holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress gives for the context's device (sevo_ctx::scratch).
constexpr size_t NOALLOC_TABLE_BYTES = (size_t)1 << 20;
static __device__ __align__(256) char scratch[NOALLOC_TABLE_BYTES];

struct sevo_ctx {
    int device = 0;
    uint64_t base_seed = 0, inst_seed = 0;
    std::string err;
    std::map<std::tuple<int, int, uint32_t>, std::unique_ptr<DevInstance>> cache;
    std::vector<DescSlot> slots;
    int next_slot = 0;
    int last_slot = -1;
    Consts consts;
    int tiles_per_block = 0;     // SEVO_TILES_PER_BLOCK override; 0 = none
    int large_points = 64;       // points per D > 120 GEMM workgroup (SEVO_LARGE_POINTS: 64 or 128)
    int tuned_tpb[2][64] = {};   // sevo_tune_evaluate's choice per (float / split-bf16 kernel, k-step
                                 // class); 0 = resident grid
    sevo::Workspace ws;
    sevo_plan *rec = nullptr;           // plan being built (calls record instead of launching)
    std::vector<hipStream_t> streams;   // internal, default priority
    std::vector<hipEvent_t> fork_ev;    // one per internal stream + the fork event
    char *scratch = nullptr;            // device address of `scratch` on this context's GPU
};

// A prepared call: plan-owned device memory and the launches to enqueue.
struct sevo_plan {
    sevo_ctx *ctx = nullptr;
    std::vector<void *> dev;
    std::vector<sevo::Launch> launches;
    int lanes = 1;
};

static std::string g_create_error;

static int fail(sevo_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_error = buf;
    return code;
}

#define HIP_TRY(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t _e = (call);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail((ctx), SEVO_EDEVICE, "%s: %s", #call, hipGetErrorString(_e));       \
    } while (0)

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int check_problem(sevo_ctx *ctx, const sevo_problem *p)
{
    if (!p) return fail(ctx, SEVO_EINVAL, "problem is NULL");
    if (p->func < 0 || p->func >= NFUNC) return fail(ctx, SEVO_EINVAL, "unknown function %d", p->func);
    if (p->dim < 2 || p->dim > MAX_DIM)
        return fail(ctx, SEVO_EINVAL, "dimension %d outside [2, %d]", p->dim, MAX_DIM);
    if (!(p->lb < p->ub) || !std::isfinite(p->lb) || !std::isfinite(p->ub))
        return fail(ctx, SEVO_EINVAL, "bounds [%g, %g] invalid", p->lb, p->ub);
    return SEVO_OK;
}

int upload_instance(sevo_ctx *ctx, DevInstance &I)
{
    const int D = I.dim;
    const int RT = rt_of(D), KS = ks_of(D), K32 = ks32_of(D);
    std::vector<float> frag((size_t)RT * KS * 64, 0.f);
    for (int rt = 0; rt < RT; ++rt)
        for (int ks = 0; ks < KS; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int r = rt * 16 + (l & 15), c = ks * 4 + (l >> 4);
                if (r < D && c < D) frag[((size_t)rt * KS + ks) * 64 + l] = (float)I.M[(size_t)r * D + c];
            }
    std::vector<float> tab((size_t)RT * 16, 0.f);
    for (int r = 0; r < D; ++r) {
        if (I.func == ELLIPSOID) tab[r] = (float)std::pow(10.0, 6.0 * r / (double)(D - 1));
        else if (I.func == GRIEWANK) tab[r] = (float)(1.0 / (2.0 * M_PI * std::sqrt((double)(r + 1))));
    }
    // bf16 terms hi, mid, lo of each float of M (hi + mid + lo is the float
    // exactly) in the A-operand order of the 16x16x32 bf16 MFMA (lane l
    // holds row l % 16 and eight k-slots 8 (l / 16) + e), term blocks
    // [RT][steps][64][8] one after another.
    // D > 120 (the tiled GEMM): step kk, slot e is column 32 kk + 8 (l / 16) + e.
    // D <= 120 (the small path): over the KS / 8 whole steps; step s, slot e
    // is column 4 (8 s + e) + l / 16, the column the float path's k-step
    // 8 s + e gives lane group l / 16.
    auto to_bf16 = [](float f) -> uint16_t {     // round to nearest even
        uint32_t u;
        std::memcpy(&u, &f, 4);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    };
    auto from_bf16 = [](uint16_t h) -> float {
        uint32_t u = (uint32_t)h << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    };
    const bool small = D <= SMALL_D_MAX;
    const int terms = 3;
    const int steps = small ? KS / 8 : K32;
    const size_t block = (size_t)RT * steps * 64 * 8;
    std::vector<uint16_t> bf(std::max<size_t>(terms * block, 8), 0);
    for (int rt = 0; rt < RT; ++rt)
        for (int kk = 0; kk < steps; ++kk)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 8; ++e) {
                    const int r = rt * 16 + (l & 15);
                    const int c = small ? 4 * (8 * kk + e) + (l >> 4) : kk * 32 + (l >> 4) * 8 + e;
                    float f = 0.f;
                    if (r < D && c < D) f = (float)I.M[(size_t)r * D + c];
                    const size_t at = (((size_t)rt * steps + kk) * 64 + l) * 8 + e;
                    for (int t = 0; t < terms; ++t) {
                        const uint16_t h = to_bf16(f);
                        bf[t * block + at] = h;
                        f -= from_bf16(h);   // exact
                    }
                }
    HIP_TRY(ctx, hipMalloc(&I.d_o, sizeof(double) * D));
    HIP_TRY(ctx, hipMalloc(&I.d_M64, sizeof(double) * (size_t)D * D));
    HIP_TRY(ctx, hipMalloc(&I.d_Mfrag, sizeof(float) * frag.size()));
    HIP_TRY(ctx, hipMalloc(&I.d_tab, sizeof(float) * tab.size()));
    HIP_TRY(ctx, hipMalloc(&I.d_Mbf, sizeof(uint16_t) * bf.size()));
    HIP_TRY(ctx, hipMemcpy(I.d_o, I.o.data(), sizeof(double) * D, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(I.d_M64, I.M.data(), sizeof(double) * (size_t)D * D, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(I.d_Mfrag, frag.data(), sizeof(float) * frag.size(), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(I.d_tab, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(I.d_Mbf, bf.data(), sizeof(uint16_t) * bf.size(), hipMemcpyHostToDevice));
    return SEVO_OK;
}

void free_instance(DevInstance &I)
{
    (void)hipFree(I.d_o);
    (void)hipFree(I.d_M64);
    (void)hipFree(I.d_Mfrag);
    (void)hipFree(I.d_tab);
    (void)hipFree(I.d_Mbf);
    I.d_o = I.d_M64 = nullptr;
    I.d_Mfrag = I.d_tab = nullptr;
    I.d_Mbf = nullptr;
}

int get_instance(sevo_ctx *ctx, const sevo_problem *p, uint32_t inst, DevInstance **out)
{
    auto key = std::make_tuple((int)p->func, (int)p->dim, inst);
    auto itr = ctx->cache.find(key);
    if (itr != ctx->cache.end()) { *out = itr->second.get(); return SEVO_OK; }
    auto I = std::make_unique<DevInstance>();
    I->func = p->func;
    I->dim = p->dim;
    generate_instance(p->func, p->dim, inst, ctx->inst_seed, I->o, I->M);
    int rc = upload_instance(ctx, *I);
    if (rc != SEVO_OK) { free_instance(*I); return rc; }
    *out = I.get();
    ctx->cache.emplace(key, std::move(I));
    return SEVO_OK;
}

// Stage bytes in device memory.  Slots rotate; a slot is rewritten only
// after the kernels that read it have finished.  Content equal to a slot that
// is still valid is reused in place (read-only), with no copy.
int stage_bytes(sevo_ctx *ctx, const std::vector<char> &blob, hipStream_t stream, const void **d_out,
                int *slot_out)
{
    const size_t n = blob.size();
    if (ctx->rec) {   // building a plan: the table gets device memory of its own
        void *d = nullptr;
        int rc = sevo::plan_alloc(ctx, n, &d);
        if (rc) return rc;
        HIP_TRY(ctx, hipMemcpy(d, blob.data(), n, hipMemcpyHostToDevice));
        *d_out = d;
        *slot_out = -1;
        return SEVO_OK;
    }
    for (int k = 0; k < (int)ctx->slots.size(); ++k) {
        DescSlot &s = ctx->slots[k];
        if (s.used == n && s.valid && std::memcmp(s.h, blob.data(), n) == 0) {
            // a reader on another stream first waits for the latest reader,
            // which ran after the copy on its own stream; the event it then
            // records (finish_slot) completes after every earlier reader
            if (s.stream != stream) HIP_TRY(ctx, hipStreamWaitEvent(stream, s.done, 0));
            *d_out = s.d;
            *slot_out = k;
            return SEVO_OK;
        }
    }
    const int idx = ctx->next_slot;
    ctx->next_slot = (ctx->next_slot + 1) % (int)ctx->slots.size();
    DescSlot &s = ctx->slots[idx];
    HIP_TRY(ctx, hipEventSynchronize(s.done));
    if (s.cap < n) {
        (void)hipHostFree(s.h);
        (void)hipFree(s.d);
        s.h = nullptr; s.d = nullptr; s.cap = 0;
        const size_t cap = std::max<size_t>(n, 64 * 1024);
        HIP_TRY(ctx, hipHostMalloc((void **)&s.h, cap, hipHostMallocDefault));
        HIP_TRY(ctx, hipMalloc((void **)&s.d, cap));
        s.cap = cap;
    }
    s.valid = false;
    std::memcpy(s.h, blob.data(), n);
    s.used = n;
    HIP_TRY(ctx, hipMemcpyAsync(s.d, s.h, n, hipMemcpyHostToDevice, stream));
    s.valid = true;
    *d_out = s.d;
    *slot_out = idx;
    return SEVO_OK;
}

int finish_slot_impl(sevo_ctx *ctx, int slot, hipStream_t stream)
{
    if (slot < 0) return SEVO_OK;   // plan-owned table
    HIP_TRY(ctx, hipEventRecord(ctx->slots[slot].done, stream));
    ctx->slots[slot].stream = stream;
    return SEVO_OK;
}

// Workgroups of a small-D launch: as many as the GPU holds at once, or
// tiles / tpb for a tiles-per-workgroup choice (the SEVO_TILES_PER_BLOCK
// override, else the autotuner's), never more than there are tiles.
int small_grid(sevo_ctx *ctx, int ks, bool bf16, int tiles)
{
    static std::map<int, int> resident;
    const int key = ks * 2 + (bf16 ? 1 : 0);
    auto itr = resident.find(key);
    if (itr == resident.end()) itr = resident.emplace(key, small_resident_blocks(ks, bf16)).first;
    long g = itr->second;
    const int tpb =
        ctx->tiles_per_block > 0 ? ctx->tiles_per_block : (ks < 64 ? ctx->tuned_tpb[bf16 ? 1 : 0][ks] : 0);
    if (tpb > 0) g = (tiles + tpb - 1) / tpb;
    return (int)std::max<long>(1, std::min<long>(g, tiles));
}

}  // namespace

// An evaluation table: item descriptors followed by the logical block ->
// item map.
static std::vector<char> table_blob(const std::vector<EvalDesc> &descs)
{
    std::vector<char> blob(descs.size() * sizeof(EvalDesc));
    std::memcpy(blob.data(), descs.data(), blob.size());
    int total = 0;
    for (const auto &d : descs) total = std::max(total, d.block0 + d.nblocks);
    std::vector<int32_t> map(total, 0);
    for (size_t i = 0; i < descs.size(); ++i)
        for (int b = 0; b < descs[i].nblocks; ++b) map[descs[i].block0 + b] = (int32_t)i;
    const size_t off = blob.size();
    blob.resize(off + map.size() * sizeof(int32_t));
    if (!map.empty()) std::memcpy(blob.data() + off, map.data(), map.size() * sizeof(int32_t));
    return blob;
}

size_t sevo::large_partial_floats(const std::vector<EvalDesc> &items, int precision)
{
    size_t n = 0;
    for (const auto &d : items)
        if (precision != SEVO_FP64 && d.n > 0 && d.dim > SMALL_D_MAX)
            n += (size_t)((d.dim + LARGE_ROWS - 1) / LARGE_ROWS) * d.n * 8;
    return n;
}

size_t sevo::large_operand_bytes(const std::vector<EvalDesc> &items, int precision)
{
    size_t n = 0;
    if (precision == SEVO_FP64) return 0;
    for (const auto &d : items)
        if (d.n > 0 && d.dim > SMALL_D_MAX)
            n += (size_t)(large_operand_size(precision == SEVO_SPLIT_BF16) * large_npad(d.n) * large_kpad(d.dim));
    return n;
}

int sevo::prepare_eval(sevo_ctx *ctx, std::vector<EvalDesc> items, int precision, float *part, void *opnd,
                       std::vector<PreparedLaunch> &out)
{
    // group: FP64 -> one launch; FP32/BF16 small D -> one launch per KS;
    // large D -> one launch pair (partial sums per 128-row block of z, then
    // a combine pass)
    std::map<int, std::vector<EvalDesc>> small;
    std::vector<EvalDesc> f64, large;
    for (const auto &d : items) {
        if (d.n <= 0) continue;
        if (precision == SEVO_FP64) f64.push_back(d);
        else if (d.dim <= SMALL_D_MAX) small[ks_of(d.dim)].push_back(d);
        else large.push_back(d);
    }
    // (the launches stay in order on the caller's stream: measured, running
    // the classes concurrently on internal streams was slower)
    for (auto &kv : small) {
        std::vector<EvalDesc> &v = kv.second;
        const int ks = kv.first;
        const bool bf16 = precision == SEVO_SPLIT_BF16 && small_bf16_class(ks);
        const int tp = small_tile_points(ks, bf16);
        int tiles = 0;
        for (auto &d : v) {
            d.block0 = tiles;                       // first tile of the item
            d.nblocks = (d.n + tp - 1) / tp;        // tiles of the item
            tiles += d.nblocks;
        }
        const int grid = small_grid(ctx, ks, bf16, tiles);
        out.push_back({Launch{L_SMALL, nullptr, (int)v.size(), ks, tiles, grid, bf16, false, 0, 0, 0},
                       table_blob(v)});
    }
    if (!f64.empty()) {
        int blocks = 0;
        for (auto &d : f64) {
            d.block0 = blocks;
            d.nblocks = (d.n + F64_POINTS - 1) / F64_POINTS;
            blocks += d.nblocks;
        }
        out.push_back({Launch{L_F64, nullptr, (int)f64.size(), 0, blocks, 0, false, false, 0, 0, 0},
                       table_blob(f64)});
    }
    if (!large.empty()) {
        if (!part) return set_error(ctx, SEVO_EINVAL, "no partial-sum buffer for a large evaluation");
        // operands first: blocks of 64 points x 32 coordinates over the
        // padded tile grid
        if (!opnd) return set_error(ctx, SEVO_EINVAL, "no operand buffer for a large evaluation");
        const bool bf16 = precision == SEVO_SPLIT_BF16;
        int oblocks = 0;
        size_t ooff = 0;
        for (auto &d : large) {
            const int64_t np = large_npad(d.n), kp = large_kpad(d.dim);
            d.opnd = static_cast<char *>(opnd) + ooff;
            ooff += (size_t)(large_operand_size(bf16) * np * kp);
            d.block0 = oblocks;
            d.nblocks = (int)((np / OPERAND_POINTS) * (kp / OPERAND_K));
            oblocks += d.nblocks;
        }
        out.push_back({Launch{L_OPERANDS, nullptr, (int)large.size(), 0, oblocks, 0, bf16, false, 0, 0, 0},
                       table_blob(large)});
        int blocks = 0;
        size_t off = 0;
        for (auto &d : large) {
            d.rb = (d.dim + LARGE_ROWS - 1) / LARGE_ROWS;
            d.block0 = blocks;
            d.nblocks = d.rb * ((d.n + ctx->large_points - 1) / ctx->large_points);
            blocks += d.nblocks;
            d.part = part + off;
            off += (size_t)d.rb * d.n * 8;
        }
        out.push_back({Launch{L_LARGE, nullptr, (int)large.size(), ctx->large_points, blocks, 0,
                              precision == SEVO_SPLIT_BF16,
                              false, 0, 0, 0},
                       table_blob(large)});
        // combine: one thread per point, blocks of 256 points
        int cblocks = 0;
        for (auto &d : large) {
            d.block0 = cblocks;
            d.nblocks = (d.n + 255) / 256;
            cblocks += d.nblocks;
        }
        out.push_back({Launch{L_COMBINE, nullptr, (int)large.size(), 0, cblocks, 0, false, false, 0, 0, 0},
                       table_blob(large)});
    }
    return SEVO_OK;
}

// Evaluate a list of (item, instance) pairs already validated: tables staged
// in the rotating slots, launches enqueued (or recorded by a plan).
int sevo::eval_items(sevo_ctx *ctx, const std::vector<std::pair<EvalDesc, int>> &items,
                     int precision, hipStream_t stream)
{
    std::vector<EvalDesc> v;
    v.reserve(items.size());
    for (const auto &pr : items) v.push_back(pr.first);
    float *part = nullptr;
    const size_t pf = large_partial_floats(v, precision), sb = large_operand_bytes(v, precision);
    void *opnd = nullptr;
    int rc;
    if (pf && (rc = ctx->ws.get(ctx, WS_PARTIAL, pf * sizeof(float), (void **)&part))) return rc;
    if (sb && (rc = ctx->ws.get(ctx, WS_OPERANDS, sb, &opnd))) return rc;
    std::vector<PreparedLaunch> pl;
    if ((rc = prepare_eval(ctx, std::move(v), precision, part, opnd, pl))) return rc;
    for (auto &p : pl) {
        const void *d = nullptr;
        int slot;
        if ((rc = stage_bytes(ctx, p.table, stream, &d, &slot))) return rc;
        p.L.d = d;
        if ((rc = emit_launch(ctx, p.L, stream))) return rc;
        if ((rc = finish_slot_impl(ctx, slot, stream))) return rc;
    }
    return SEVO_OK;
}

// ---------------------------------------------------------------------------
// Workspace

int sevo::Workspace::get(sevo_ctx *ctx, int which, size_t bytes, void **out)
{
    if (ctx->rec) return plan_alloc(ctx, std::max<size_t>(bytes, 256), out);   // a plan's own workspace
    Buf &b = bufs[which];
    if (b.bytes < bytes) {
        if (b.ptr) {
            HIP_TRY(ctx, hipDeviceSynchronize());
            (void)hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        const size_t cap = std::max<size_t>(bytes, 1 << 20);
        HIP_TRY(ctx, hipMalloc(&b.ptr, cap));
        b.bytes = cap;
    }
    *out = b.ptr;
    return SEVO_OK;
}

void sevo::Workspace::release()
{
    for (auto &b : bufs) {
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
}

int sevo::set_error(sevo_ctx *ctx, int code, const char *msg)
{
    return fail(ctx, code, "%s", msg);
}

int sevo::lookup_instance(sevo_ctx *ctx, const sevo_problem *p, uint32_t inst, InstanceView *out)
{
    DevInstance *I = nullptr;
    int rc = get_instance(ctx, p, inst, &I);
    if (rc) return rc;
    out->o = I->d_o;
    out->M64 = I->d_M64;
    out->Mfrag = I->d_Mfrag;
    out->tab = I->d_tab;
    out->Mbf = I->d_Mbf;
    return SEVO_OK;
}

int sevo::stage_blob(sevo_ctx *ctx, const std::vector<char> &blob, hipStream_t stream,
                     const void **d_out, int *slot_out)
{
    return stage_bytes(ctx, blob, stream, d_out, slot_out);
}

int sevo::finish_slot(sevo_ctx *ctx, int slot, hipStream_t stream)
{
    return finish_slot_impl(ctx, slot, stream);
}

static int ensure_streams(sevo_ctx *ctx, int n)
{
    while ((int)ctx->streams.size() < n) {
        hipStream_t s;
        HIP_TRY(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ctx->streams.push_back(s);
    }
    while ((int)ctx->fork_ev.size() < n + 1) {
        hipEvent_t e;
        HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->fork_ev.push_back(e);
    }
    return SEVO_OK;
}

int sevo::fork_streams(sevo_ctx *ctx, hipStream_t parent, int n, hipStream_t *out)
{
    int rc = ensure_streams(ctx, n);
    if (rc) return rc;
    HIP_TRY(ctx, hipEventRecord(ctx->fork_ev[n], parent));
    for (int k = 0; k < n; ++k) {
        HIP_TRY(ctx, hipStreamWaitEvent(ctx->streams[k], ctx->fork_ev[n], 0));
        out[k] = ctx->streams[k];
    }
    return SEVO_OK;
}

int sevo::join_streams(sevo_ctx *ctx, hipStream_t parent, int n, const hipStream_t *streams)
{
    for (int k = 0; k < n; ++k) {
        HIP_TRY(ctx, hipEventRecord(ctx->fork_ev[k], streams[k]));
        HIP_TRY(ctx, hipStreamWaitEvent(parent, ctx->fork_ev[k], 0));
    }
    return SEVO_OK;
}

sevo::DeviceScope::DeviceScope(sevo_ctx *ctx)
{
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
}

sevo::DeviceScope::~DeviceScope()
{
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

sevo_plan *sevo::ctx_recording(sevo_ctx *ctx) { return ctx->rec; }

int sevo::plan_alloc(sevo_ctx *ctx, size_t bytes, void **out)
{
    void *d = nullptr;
    HIP_TRY(ctx, hipMalloc(&d, std::max<size_t>(bytes, 16)));
    ctx->rec->dev.push_back(d);
    *out = d;
    return SEVO_OK;
}

static hipError_t exec_launch(sevo_ctx *ctx, const sevo::Launch &L, hipStream_t s)
{
    using namespace sevo;
    switch (L.kind) {
    case L_SMALL:
        return launch_eval_small((const EvalDesc *)L.d, L.n, L.ks, L.total, L.grid, L.flag, ctx->consts, s);
    case L_F64: return launch_eval_f64((const EvalDesc *)L.d, L.n, L.total, ctx->consts, s);
    case L_LARGE: return launch_eval_large((const EvalDesc *)L.d, L.n, L.total, L.flag, L.ks, ctx->consts, s);
    case L_COMBINE: return launch_eval_large_combine((const EvalDesc *)L.d, L.n, L.total, ctx->consts, s);
    case L_OPERANDS: return launch_eval_operands((const EvalDesc *)L.d, L.n, L.total, L.flag, s);
    case L_RUN: return exec_run_launch(L, s, fold_seed(ctx->base_seed), ctx->consts);
    case L_CSO: return exec_cso_launch(L, s, fold_seed(ctx->base_seed), ctx->consts);
    default: return hipErrorInvalidValue;
    }
}

int sevo::emit_launch(sevo_ctx *ctx, const Launch &L, hipStream_t stream)
{
    if (ctx->rec) {
        ctx->rec->launches.push_back(L);
        ctx->rec->lanes = std::max(ctx->rec->lanes, L.lane + 1);
        return SEVO_OK;
    }
    HIP_TRY(ctx, exec_launch(ctx, L, stream));
    return SEVO_OK;
}

static void free_plan(sevo_plan *p)
{
    if (!p) return;
    if (!p->dev.empty()) (void)hipDeviceSynchronize();
    for (void *d : p->dev) (void)hipFree(d);
    delete p;
}

int sevo::plan_begin(sevo_ctx *ctx)
{
    if (ctx->rec) return fail(ctx, SEVO_ESTATE, "a plan is already being built on this context");
    ctx->rec = new sevo_plan;
    ctx->rec->ctx = ctx;
    return SEVO_OK;
}

int sevo::plan_finish(sevo_ctx *ctx, int rc, sevo_plan **out)
{
    sevo_plan *p = ctx->rec;
    ctx->rec = nullptr;
    // create the internal streams now: launching the plan creates nothing
    if (rc == SEVO_OK && p && p->lanes > 1) rc = ensure_streams(ctx, p->lanes);
    if (rc != SEVO_OK) {
        free_plan(p);
        *out = nullptr;
        return rc;
    }
    *out = p;
    return SEVO_OK;
}

const Consts &sevo::ctx_consts(sevo_ctx *ctx) { return ctx->consts; }
uint32_t sevo::ctx_seed32(sevo_ctx *ctx) { return fold_seed(ctx->base_seed); }
Workspace &sevo::ctx_ws(sevo_ctx *ctx) { return ctx->ws; }

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int sevo_create(sevo_ctx **out, int32_t hip_device, uint64_t base_seed, uint64_t instance_seed)
{
    if (!out) return fail(nullptr, SEVO_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(nullptr, SEVO_EDEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= n)
        return fail(nullptr, SEVO_EINVAL, "device %d not in [0, %d)", hip_device, n);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, hip_device);
    if (e != hipSuccess)
        return fail(nullptr, SEVO_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, SEVO_EUNSUPPORTED, "device %d is %s; this library is built for gfx950",
                    hip_device, prop.gcnArchName);
    auto ctx = std::make_unique<sevo_ctx>();
    ctx->device = hip_device;
    ctx->base_seed = base_seed;
    ctx->inst_seed = instance_seed;
    ctx->consts = make_consts();
    if (const char *e = std::getenv("SEVO_TILES_PER_BLOCK")) ctx->tiles_per_block = std::atoi(e);
    if (const char *e = std::getenv("SEVO_LARGE_POINTS")) ctx->large_points = std::atoi(e) == 128 ? 128 : 64;
    DeviceGuard g(hip_device);
    e = hipGetSymbolAddress((void **)&ctx->scratch, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return fail(nullptr, SEVO_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    ctx->slots.resize(16);
    for (auto &s : ctx->slots) {
        e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e != hipSuccess)
            return fail(nullptr, SEVO_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    *out = ctx.release();
    return SEVO_OK;
}

int sevo_destroy(sevo_ctx *ctx)
{
    if (!ctx) return SEVO_OK;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &kv : ctx->cache) free_instance(*kv.second);
        for (auto &s : ctx->slots) {
            (void)hipHostFree(s.h);
            (void)hipFree(s.d);
            if (s.done) (void)hipEventDestroy(s.done);
        }
        ctx->ws.release();
        sevo::release_state(ctx);
        for (auto s : ctx->streams) (void)hipStreamDestroy(s);
        for (auto e : ctx->fork_ev) (void)hipEventDestroy(e);
    }
    delete ctx;
    return SEVO_OK;
}

const char *sevo_last_error(const sevo_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int sevo_sync(sevo_ctx *ctx, void *stream)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(ctx, hipGetLastError());
    return SEVO_OK;
}

int sevo_instance(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance, double *o_host,
                  double *M_host)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    int rc = check_problem(ctx, prob);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    DevInstance *I = nullptr;
    if ((rc = get_instance(ctx, prob, instance, &I))) return rc;
    if (o_host) std::memcpy(o_host, I->o.data(), sizeof(double) * I->dim);
    if (M_host) std::memcpy(M_host, I->M.data(), sizeof(double) * (size_t)I->dim * I->dim);
    return SEVO_OK;
}

int sevo_generate_instance(int32_t func, int32_t dim, uint32_t instance, uint64_t instance_seed,
                           double *o_host, double *M_host)
{
    sevo_problem p{func, dim, -1.0, 1.0, 0.0};
    int rc = check_problem(nullptr, &p);
    if (rc) return rc;
    if (!o_host || !M_host) return fail(nullptr, SEVO_EINVAL, "o and M must be given");
    std::vector<double> o, M;
    generate_instance(func, dim, instance, instance_seed, o, M);
    std::memcpy(o_host, o.data(), sizeof(double) * dim);
    std::memcpy(M_host, M.data(), sizeof(double) * (size_t)dim * dim);
    return SEVO_OK;
}

int sevo_set_instance(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance,
                      const double *o_host, const double *M_host)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    int rc = check_problem(ctx, prob);
    if (rc) return rc;
    if (!o_host || !M_host) return fail(ctx, SEVO_EINVAL, "o and M must be given");
    for (int j = 0; j < prob->dim; ++j)
        if (!std::isfinite(o_host[j])) return fail(ctx, SEVO_EINVAL, "o[%d] is not finite", j);
    for (size_t j = 0; j < (size_t)prob->dim * prob->dim; ++j)
        if (!std::isfinite(M_host[j])) return fail(ctx, SEVO_EINVAL, "M[%zu] is not finite", j);
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, hipDeviceSynchronize());   // the old copy may still be read
    auto key = std::make_tuple((int)prob->func, (int)prob->dim, instance);
    auto itr = ctx->cache.find(key);
    if (itr != ctx->cache.end()) {
        free_instance(*itr->second);
        ctx->cache.erase(itr);
    }
    ctx->last_slot = -1;   // cached descriptor tables may point at the old copy
    for (auto &sl : ctx->slots) sl.valid = false;
    auto I = std::make_unique<DevInstance>();
    I->func = prob->func;
    I->dim = prob->dim;
    I->o.assign(o_host, o_host + prob->dim);
    I->M.assign(M_host, M_host + (size_t)prob->dim * prob->dim);
    if ((rc = upload_instance(ctx, *I))) { free_instance(*I); return rc; }
    ctx->cache.emplace(key, std::move(I));
    return SEVO_OK;
}

static int check_precision(sevo_ctx *ctx, int precision)
{
    if (precision != SEVO_FP64 && precision != SEVO_FP32 && precision != SEVO_SPLIT_BF16)
        return fail(ctx, SEVO_EINVAL, "unknown precision %d", precision);
    return SEVO_OK;
}

static int build_items(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items,
                       std::vector<std::pair<EvalDesc, int>> &v)
{
    int rc;
    v.reserve(n_items);
    for (int i = 0; i < n_items; ++i) {
        const sevo_eval_item &it = items[i];
        if ((rc = check_problem(ctx, &it.prob))) return rc;
        if (it.n < 0) return fail(ctx, SEVO_EINVAL, "item %d: n = %d", i, it.n);
        if (it.n == 0) continue;
        if (it.ld < it.n) return fail(ctx, SEVO_EINVAL, "item %d: ld %lld < n %d", i, (long long)it.ld, it.n);
        if (it.ld > MAX_LD) return fail(ctx, SEVO_EINVAL, "item %d: ld %lld > 2^28", i, (long long)it.ld);
        if (!it.x || !it.err_out) return fail(ctx, SEVO_EINVAL, "item %d: null buffer", i);
        DevInstance *I = nullptr;
        if ((rc = get_instance(ctx, &it.prob, it.instance, &I))) return rc;
        EvalDesc d{};
        d.x = it.x;
        d.err = it.err_out;
        d.o = I->d_o;
        d.Mfrag = I->d_Mfrag;
        d.tab = I->d_tab;
        d.M64 = I->d_M64;
        d.Mbf = I->d_Mbf;
        d.ld = it.ld;
        d.n = it.n;
        d.func = it.prob.func;
        d.dim = it.prob.dim;
        v.emplace_back(d, i);
    }
    return SEVO_OK;
}

int sevo_evaluate_batch(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items,
                        int32_t precision, void *stream)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    int rc = check_precision(ctx, precision);
    if (rc) return rc;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, SEVO_EINVAL, "bad item list");
    DeviceGuard g(ctx->device);
    std::vector<std::pair<EvalDesc, int>> v;
    if ((rc = build_items(ctx, items, n_items, v))) return rc;
    return eval_items(ctx, v, precision, (hipStream_t)stream);
}

int sevo_evaluate_batch_noalloc(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items,
                                int32_t precision, void *stream)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    int rc = check_precision(ctx, precision);
    if (rc) return rc;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, SEVO_EINVAL, "bad item list");
    DeviceGuard g(ctx->device);
    std::vector<EvalDesc> v;
    v.reserve(n_items);
    for (int i = 0; i < n_items; ++i) {
        const sevo_eval_item &it = items[i];
        if ((rc = check_problem(ctx, &it.prob))) return rc;
        if (it.n < 0) return fail(ctx, SEVO_EINVAL, "item %d: n = %d", i, it.n);
        if (it.n == 0) continue;
        if (it.ld < it.n) return fail(ctx, SEVO_EINVAL, "item %d: ld %lld < n %d", i, (long long)it.ld, it.n);
        if (it.ld > MAX_LD) return fail(ctx, SEVO_EINVAL, "item %d: ld %lld > 2^28", i, (long long)it.ld);
        if (!it.x || !it.err_out) return fail(ctx, SEVO_EINVAL, "item %d: null buffer", i);
        if (precision != SEVO_FP64 && it.prob.dim > SMALL_D_MAX)
            return fail(ctx, SEVO_EUNSUPPORTED,
                        "item %d: D = %d > %d needs the GEMM workspace (sevo_evaluate_batch)", i, it.prob.dim,
                        SMALL_D_MAX);
        // no instance is made here: that would allocate
        auto itr = ctx->cache.find(std::make_tuple((int)it.prob.func, (int)it.prob.dim, it.instance));
        if (itr == ctx->cache.end())
            return fail(ctx, SEVO_ESTATE,
                        "item %d: instance %u of (func %d, D %d) is not resident; make it first "
                        "(sevo_instance or any other evaluation)", i, it.instance, it.prob.func, it.prob.dim);
        const DevInstance &I = *itr->second;
        EvalDesc d{};
        d.x = it.x;
        d.err = it.err_out;
        d.o = I.d_o;
        d.Mfrag = I.d_Mfrag;
        d.tab = I.d_tab;
        d.M64 = I.d_M64;
        d.Mbf = I.d_Mbf;
        d.ld = it.ld;
        d.n = it.n;
        d.func = it.prob.func;
        d.dim = it.prob.dim;
        v.push_back(d);
    }
    std::vector<PreparedLaunch> pl;
    if ((rc = prepare_eval(ctx, std::move(v), precision, nullptr, nullptr, pl))) return rc;
    size_t need = 0;
    for (const auto &p : pl) need += (p.table.size() + 255) & ~(size_t)255;
    if (need > NOALLOC_TABLE_BYTES)
        return fail(ctx, SEVO_EINVAL, "the call's descriptor tables take %zu bytes; the static table holds %zu",
                    need, NOALLOC_TABLE_BYTES);
    // tables into the device array, each launch after its table on the
    // caller's stream (so a later call on the same stream rewrites them only
    // after these kernels)
    size_t off = 0;
    for (auto &p : pl) {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->scratch + off, p.table.data(), p.table.size(), hipMemcpyHostToDevice,
                                    (hipStream_t)stream));
        p.L.d = ctx->scratch + off;
        if ((rc = emit_launch(ctx, p.L, (hipStream_t)stream))) return rc;
        off += (p.table.size() + 255) & ~(size_t)255;
    }
    return SEVO_OK;
}

int sevo_tune_evaluate(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items, int32_t precision,
                       void *stream, int32_t *chosen)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    int rc = check_precision(ctx, precision);
    if (rc) return rc;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, SEVO_EINVAL, "bad item list");
    DeviceGuard g(ctx->device);
    std::vector<std::pair<EvalDesc, int>> v;
    if ((rc = build_items(ctx, items, n_items, v))) return rc;
    if (chosen)
        for (int k = 0; k < 64; ++k) chosen[k] = -1;
    if (precision == SEVO_FP64) return SEVO_OK;   // one thread per point: nothing to choose
    std::map<int, std::vector<std::pair<EvalDesc, int>>> by_ks;
    for (const auto &pr : v)
        if (pr.first.dim <= SMALL_D_MAX) by_ks[ks_of(pr.first.dim)].push_back(pr);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    const int saved_override = ctx->tiles_per_block;
    ctx->tiles_per_block = 0;
    // candidates: fixed tiles per workgroup and the resident grid (0); every
    // candidate computes the same values, so the outputs are simply rewritten.
    // Within 2 % of the fastest the earliest candidate is kept: fewer tiles
    // per workgroup move fewer bytes (measured at D = 100: one tile 1.03 x the
    // algorithmic bytes, three 1.19 x, the resident grid 1.20 x), and the
    // pick no longer follows timing noise between shapes that close.
    const int cand[] = {1, 2, 3, 4, 6, 8, 0};
    for (auto &kv : by_ks) {
        const int ks = kv.first;
        // the table of the kernel this precision runs for the class
        int *tuned = &ctx->tuned_tpb[precision == SEVO_SPLIT_BF16 && small_bf16_class(ks) ? 1 : 0][ks];
        float ms_of[sizeof(cand) / sizeof(cand[0])] = {};
        int nc = 0;
        for (int c : cand) {
            *tuned = c;
            if ((rc = eval_items(ctx, kv.second, precision, st))) break;   // warm-up
            float ms_min = 0.f;
            for (int rep = 0; rep < 3 && !rc; ++rep) {
                if (hipEventRecord(e0, st) != hipSuccess) rc = fail(ctx, SEVO_EDEVICE, "event record failed");
                if (!rc) rc = eval_items(ctx, kv.second, precision, st);
                if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = fail(ctx, SEVO_EDEVICE, "event record failed");
                if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(ctx, SEVO_EDEVICE, "event sync failed");
                float ms = 0.f;
                if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(ctx, SEVO_EDEVICE, "event time failed");
                if (!rc && (rep == 0 || ms < ms_min)) ms_min = ms;
            }
            if (rc) break;
            ms_of[nc++] = ms_min;
        }
        if (rc) break;
        float fastest = ms_of[0];
        for (int q = 1; q < nc; ++q) fastest = std::min(fastest, ms_of[q]);
        int best_tpb = cand[0];
        for (int q = 0; q < nc; ++q)
            if (ms_of[q] <= 1.02f * fastest) { best_tpb = cand[q]; break; }
        *tuned = best_tpb;
        if (chosen) chosen[ks] = best_tpb;
    }
    ctx->tiles_per_block = saved_override;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int sevo_plan_evaluate(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items, int32_t precision,
                       sevo_plan **out)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!out) return fail(ctx, SEVO_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_precision(ctx, precision);
    if (rc) return rc;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, SEVO_EINVAL, "bad item list");
    DeviceGuard g(ctx->device);
    std::vector<std::pair<EvalDesc, int>> v;
    if ((rc = build_items(ctx, items, n_items, v))) return rc;   // instances made before recording
    if ((rc = plan_begin(ctx))) return rc;
    rc = eval_items(ctx, v, precision, nullptr);
    return plan_finish(ctx, rc, out);
}

int sevo_plan_launch(sevo_plan *plan, void *stream)
{
    if (!plan) return fail(nullptr, SEVO_EINVAL, "plan is NULL");
    sevo_ctx *ctx = plan->ctx;
    DeviceGuard g(ctx->device);
    const hipStream_t s = (hipStream_t)stream;
    std::vector<hipStream_t> ss(plan->lanes, s);
    int rc;
    if (plan->lanes > 1 && (rc = fork_streams(ctx, s, plan->lanes, ss.data()))) return rc;
    for (const Launch &L : plan->launches) HIP_TRY(ctx, exec_launch(ctx, L, ss[L.lane]));
    if (plan->lanes > 1) return join_streams(ctx, s, plan->lanes, ss.data());
    return SEVO_OK;
}

int sevo_plan_destroy(sevo_plan *plan)
{
    if (!plan) return SEVO_OK;
    DeviceGuard g(plan->ctx->device);
    free_plan(plan);
    return SEVO_OK;
}

int sevo_evaluate(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance, const void *x,
                  int64_t ld, int32_t n, void *err_out, int32_t precision, void *stream)
{
    if (!ctx) return fail(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!prob) return fail(ctx, SEVO_EINVAL, "problem is NULL");
    sevo_eval_item it;
    it.prob = *prob;
    it.instance = instance;
    it.n = n;
    it.ld = ld;
    it.x = x;
    it.err_out = err_out;
    return sevo_evaluate_batch(ctx, &it, 1, precision, stream);
}

}  // extern "C"
