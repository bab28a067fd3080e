// batch.cpp -- host side of the batched matcher: per-pair scratch, the work
// list of the persistent kernel (k_batch.hip), the aggregation-tile
// autotuner with its cache file, and the HIP graph that replays the launch.
#include <errno.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dco_batch.h"

namespace {

struct Tile {
    int band, dchunk;
};

}  // namespace

struct dco_batch {
    int n = 0;
    dco_params p{};
    hipStream_t stream = nullptr;     // the caller's stream
    hipStream_t cap_stream = nullptr; // private stream used for graph capture
    std::vector<BatchPair> pairs;
    std::vector<Tile> tiles;
    BatchPair* d_pairs = nullptr;
    BatchIO* d_io = nullptr;
    BatchIO* h_io = nullptr;          // pinned staging of the pointer table
    hipEvent_t io_copied = nullptr;
    bool io_pending = false;
    BatchItem* d_items = nullptr;
    int first[kBatchStages + 1] = {};  // stage s owns items [first[s], first[s + 1])
    int xsplit[kXcds + 1] = {};        // stage-2 items of each XCD
    int cus = 0;
    int per_cu[kBatchStages] = {};
    float *tabA = nullptr, *tabC = nullptr, *alpha = nullptr, *beta = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> allocs;
};

namespace {

template <class T>
dco_status balloc(dco_batch* b, T** p, size_t n) {
    DCO_TRY(dev_alloc(p, n));
    b->allocs.push_back((void*)*p);
    return DCO_OK;
}

dco_status alloc_pair(dco_batch* b, BatchPair& pr, int W, int H, int D) {
    const size_t P = (size_t)W * H, V = P * D;
    pr.W = W;
    pr.H = H;
    pr.D = D;
    pr.nstrips = (W + kStripOut - 1) / kStripOut;
    for (int v = 0; v < 2; ++v) {
        DCO_TRY(balloc(b, &pr.arms[v], P));
        DCO_TRY(balloc(b, &pr.pix[v], P));
        const dco_status s = alloc_records(&pr.rec[v], W, H);
        for (void* q : {(void*)pr.rec[v].b, (void*)pr.rec[v].c})
            if (q) b->allocs.push_back(q);
        DCO_TRY(s);
        DCO_TRY(balloc(b, &pr.agg[v], V));
        DCO_TRY(balloc(b, &pr.dint[v], P));
    }
    DCO_TRY(balloc(b, &pr.delta, P));
    return DCO_OK;
}

// Stage-ordered work list.  Stage 2 is built in pair, view, strip, band,
// disparity order (neighbouring items share inputs), cut into kXcds
// contiguous parts of about equal cost, and each part ordered longest first.
std::vector<BatchItem> make_items(std::vector<BatchPair>& pairs, int* xsplit) {
    std::vector<BatchItem> st[kBatchStages];
    for (int i = 0; i < (int)pairs.size(); ++i) {
        BatchPair& pr = pairs[i];
        const int bx = (pr.W + 63) / 64, by = (pr.H + 63) / 64;
        const int nb = (pr.H + pr.band - 1) / pr.band;
        const int nd = (pr.D + pr.dchunk - 1) / pr.dchunk;
        for (int v = 0; v < 2; ++v)
            for (int y = 0; y < by; ++y)
                for (int x = 0; x < bx; ++x) {
                    st[0].push_back(BatchItem{i, 0, v, x, y, 0});
                    st[1].push_back(BatchItem{i, 1, v, x, y, 0});
                }
        // neighbouring disparities of one strip and band next to each other:
        // the workgroups that run them at the same time share their inputs
        for (int v = 0; v < 2; ++v)
            for (int s = 0; s < pr.nstrips; ++s)
                for (int c = 0; c < nb; ++c)
                    for (int d = 0; d < nd; ++d)
                        st[2].push_back(BatchItem{i, 2, v, d * pr.dchunk, s, c});
        const int P = pr.W * pr.H;
        for (int a = 0; a < P; a += kWtaPx) st[3].push_back(BatchItem{i, 3, 0, a, 0, 0});
        for (int a = 0; a < pr.H; a += kLrRows) st[4].push_back(BatchItem{i, 4, 0, a, 0, 0});
        pr.nitems[0] = pr.nitems[1] = 2 * bx * by;
        pr.nitems[2] = 2 * nb * nd * pr.nstrips;
        pr.nitems[3] = (P + kWtaPx - 1) / kWtaPx;
        pr.nitems[4] = (pr.H + kLrRows - 1) / kLrRows;
    }
    auto cost = [&](const BatchItem& it) {
        const BatchPair& pr = pairs[it.pair];
        const int y0 = it.c * pr.band, rows = std::min(pr.H, y0 + pr.band) - y0;
        const int dn = std::min(pr.dchunk, pr.D - it.a);
        return (long long)(rows + 4 * kLMax + 2) * dn;
    };
    // stage 2 in kXcds contiguous parts of about equal cost, one per XCD
    const int s2 = (int)(st[0].size() + st[1].size());
    long long total = 0;
    for (const BatchItem& it : st[2]) total += cost(it);
    long long acc = 0;
    int x = 1;
    xsplit[0] = s2;
    for (size_t k = 0; k < st[2].size() && x < kXcds; ++k) {
        acc += cost(st[2][k]);
        while (x < kXcds && acc * kXcds >= total * x) xsplit[x++] = s2 + (int)k + 1;
    }
    while (x <= kXcds) xsplit[x++] = s2 + (int)st[2].size();
    // within each XCD's part, longest items first (stable, so the items of
    // one strip and band keep their neighbouring disparities together): the
    // part's last round then holds its shortest items instead of leaving
    // resident slots idle behind a long one
    for (int k = 0; k < kXcds; ++k)
        std::stable_sort(st[2].begin() + (xsplit[k] - s2), st[2].begin() + (xsplit[k + 1] - s2),
                         [&](const BatchItem& a, const BatchItem& b) { return cost(a) > cost(b); });
    std::vector<BatchItem> all;
    for (auto& s : st) all.insert(all.end(), s.begin(), s.end());
    return all;
}

BatchArgs make_args(const dco_batch* b) {
    BatchArgs a{};
    a.pairs = b->d_pairs;
    a.io = b->d_io;
    a.items = b->d_items;
    a.tabA = b->tabA;
    a.tabC = b->tabC;
    a.alpha = b->alpha;
    a.beta = b->beta;
    a.cw = b->p.census_w;
    a.ch = b->p.census_h;
    a.L1 = b->p.arm_L1;
    a.tau1 = b->p.arm_tau1;
    a.subpixel = b->p.subpixel;
    a.maxdiff = b->p.lr_max_diff;
    for (int x = 0; x <= kXcds; ++x) a.xsplit[x] = b->xsplit[x];
    return a;
}

// The stage kernels rely on a stage-ordered list whose per-pair, per-stage
// counts are the ones recorded in the pair descriptions.  Checked on the
// host; fills the stage offsets.
dco_status check_items(const std::vector<BatchItem>& items, const std::vector<BatchPair>& pairs,
                       int* first) {
    std::vector<int> seen(pairs.size() * kBatchStages, 0);
    int stage = 0;
    first[0] = 0;
    for (size_t k = 0; k < items.size(); ++k) {
        const BatchItem& it = items[k];
        if (it.pair < 0 || it.pair >= (int)pairs.size() || it.stage < stage ||
            it.stage >= kBatchStages) {
            dco_set_error("batch work list: item %zu out of order", k);
            return DCO_ERR_STATE;
        }
        while (stage < it.stage) first[++stage] = (int)k;
        ++seen[it.pair * kBatchStages + it.stage];
    }
    while (stage < kBatchStages) first[++stage] = (int)items.size();
    for (size_t i = 0; i < pairs.size(); ++i)
        for (int s = 0; s < kBatchStages; ++s)
            if (seen[i * kBatchStages + s] != pairs[i].nitems[s] || pairs[i].nitems[s] < 1) {
                dco_set_error("batch work list: pair %zu stage %d count mismatch", i, s);
                return DCO_ERR_STATE;
            }
    return DCO_OK;
}

// (Re)build the work list and upload pairs and items.
dco_status upload(dco_batch* b) {
    std::vector<BatchItem> items = make_items(b->pairs, b->xsplit);
    DCO_TRY(check_items(items, b->pairs, b->first));
    if (b->d_items) {
        dev_free(b->d_items);
        b->allocs.erase(std::find(b->allocs.begin(), b->allocs.end(), (void*)b->d_items));
        b->d_items = nullptr;
    }
    DCO_TRY(balloc(b, &b->d_items, items.size()));
    DCO_HIP_CHECK(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(BatchItem),
                            hipMemcpyHostToDevice));
    DCO_HIP_CHECK(hipMemcpy(b->d_pairs, b->pairs.data(), b->pairs.size() * sizeof(BatchPair),
                            hipMemcpyHostToDevice));
    return DCO_OK;
}

dco_status make_base(dco_batch* b, int n, const dco_params& p) {
    b->n = n;
    b->p = p;
    std::vector<float> tA, tC, al, be;
    build_tables(p, tA, tC, al, be);
    DCO_TRY(balloc(b, &b->tabA, tA.size()));
    DCO_TRY(balloc(b, &b->tabC, tC.size()));
    DCO_TRY(balloc(b, &b->alpha, al.size()));
    DCO_TRY(balloc(b, &b->beta, be.size()));
    DCO_HIP_CHECK(hipMemcpy(b->tabA, tA.data(), tA.size() * 4, hipMemcpyHostToDevice));
    DCO_HIP_CHECK(hipMemcpy(b->tabC, tC.data(), tC.size() * 4, hipMemcpyHostToDevice));
    DCO_HIP_CHECK(hipMemcpy(b->alpha, al.data(), al.size() * 4, hipMemcpyHostToDevice));
    DCO_HIP_CHECK(hipMemcpy(b->beta, be.data(), be.size() * 4, hipMemcpyHostToDevice));
    DCO_TRY(balloc(b, &b->d_pairs, (size_t)n));
    DCO_TRY(balloc(b, &b->d_io, (size_t)n));
    int dev = 0;
    DCO_HIP_CHECK(hipGetDevice(&dev));
    DCO_HIP_CHECK(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev));
    batch_blocks_per_cu(p.agg_iters, b->per_cu);
    b->pairs.assign(n, BatchPair{});
    b->tiles.assign(n, Tile{0, 1});
    return DCO_OK;
}

void release(dco_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->io_copied) (void)hipEventDestroy(b->io_copied);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    pinned_free(b->h_io);
    b->h_io = nullptr;
    for (void* p : b->allocs) dev_free(p);
    b->allocs.clear();
}

// Grid of each stage kernel: its items, at most the resident capacity.
hipError_t launch(const dco_batch* b, hipStream_t st) {
    int grid[kBatchStages];
    for (int s = 0; s < kBatchStages; ++s)
        grid[s] = std::max(1, std::min(b->first[s + 1] - b->first[s], b->cus * b->per_cu[s]));
    int most = 1;  // stage 2: one workgroup per item, kXcds x the largest XCD part
    for (int x = 0; x < kXcds; ++x) most = std::max(most, b->xsplit[x + 1] - b->xsplit[x]);
    grid[2] = kXcds * most;
    return launch_batch(make_args(b), b->p.agg_iters, b->first, grid, st);
}

// ---- autotuner -------------------------------------------------------------

std::string cache_path() {
    if (const char* e = getenv("DCO_AUTOTUNE_CACHE")) return e;
    const char* home = getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/dco_stereo_autotune.txt";
}

// The key names the stage-2 kernel generation too ("s2" = two disparities
// per pass), so tiles timed with another kernel are not reused.
std::string class_key(int W, int H, int D, int iters, const char* arch) {
    char buf[160];
    snprintf(buf, sizeof buf, "%dx%dx%d:%s:iters%d:s2", W, H, D, arch, iters);
    return buf;
}

// Cache format: one "key band dchunk" line per size class.
std::map<std::string, Tile> read_cache() {
    std::map<std::string, Tile> m;
    FILE* f = fopen(cache_path().c_str(), "r");
    if (!f) return m;
    char key[160];
    int band, dc;
    while (fscanf(f, "%159s %d %d", key, &band, &dc) == 3)
        if (band > 0 && dc > 0) m[key] = Tile{band, dc};
    fclose(f);
    return m;
}

// Creates every missing directory of `path` (mkdir(2) only: no child process).
bool make_dirs(const std::string& path) {
    for (size_t i = 1; i <= path.size(); ++i) {
        if (i < path.size() && path[i] != '/') continue;
        const std::string part = path.substr(0, i);
        if (mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) return false;
    }
    return true;
}

void write_cache(const std::map<std::string, Tile>& m) {
    const std::string path = cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0 && !make_dirs(path.substr(0, slash))) return;
    FILE* f = fopen(path.c_str(), "w");
    if (!f) return;
    for (auto& kv : m) fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.band, kv.second.dchunk);
    fclose(f);
}

// Disparity chunks to time, with full-height bands.  A batch fills the GPU
// with items already, and every band of a split would start 2 L1 + 1 rows
// early: on the 32-pair workload, tiles with bands of H / 2 chosen on copies
// of one size class made the batch 3 % slower than full-height items.  With
// two aggregation stages the kernel takes two disparities per pass, so
// chunks are even (a range of one disparity keeps a chunk of one).
std::vector<Tile> candidates(int H, int D, int iters) {
    std::vector<Tile> out;
    const int chunks1[] = {1, 2, 4}, chunks2[] = {2, 4, 8};
    const int* chunks = iters == 2 ? chunks2 : chunks1;
    for (int k = 0; k < 3; ++k) {
        const int dc = chunks[k];
        if (dc <= D || (k == 0 && D < dc)) out.push_back(Tile{H, std::min(dc, D)});
    }
    return out;
}

// Times every candidate tile on copies of a synthetic pair of one size class.
// There are enough copies that the untiled cost + aggregation stage has about
// four times as many items as resident workgroups, as in a full batch:
// timed alone, one small pair would favour short bands for parallelism that
// a batch gets from its other pairs anyway.
dco_status tune_class(const dco_params& p, int W, int H, int D, hipStream_t st, Tile* best) {
    dco_batch tb;
    dco_status s = make_base(&tb, 1, p);
    int copies = 1;
    if (s == DCO_OK) {
        const int nstrips = (W + kStripOut - 1) / kStripOut;
        const long long slots = (long long)tb.cus * std::max(1, tb.per_cu[2]);
        copies = (int)std::min<long long>(16, std::max<long long>(
                                                   1, (4 * slots + 2LL * nstrips * D - 1) /
                                                          (2LL * nstrips * D)));
        release(&tb);
        tb = dco_batch{};
        s = make_base(&tb, copies, p);
    }
    for (int i = 0; i < copies && s == DCO_OK; ++i) s = alloc_pair(&tb, tb.pairs[i], W, H, D);
    uint8_t *L = nullptr, *R = nullptr;
    if (s == DCO_OK) s = balloc(&tb, &L, (size_t)W * H * 3);
    if (s == DCO_OK) s = balloc(&tb, &R, (size_t)W * H * 3);
    float* disp = nullptr;
    uint8_t* valid = nullptr;
    if (s == DCO_OK) s = balloc(&tb, &disp, (size_t)W * H);
    if (s == DCO_OK) s = balloc(&tb, &valid, (size_t)W * H);
    if (s != DCO_OK) {
        release(&tb);
        return s;
    }
    // a seeded noise pair: right = left shifted by D / 2
    std::vector<uint8_t> img((size_t)W * H * 3), img2((size_t)W * H * 3);
    uint32_t x = 12345u;
    for (auto& v : img) {
        x = x * 1664525u + 1013904223u;
        v = (uint8_t)(x >> 24);
    }
    for (int y = 0; y < H; ++y)
        for (int c = 0; c < W; ++c)
            for (int k = 0; k < 3; ++k)
                img2[((size_t)y * W + c) * 3 + k] =
                    img[((size_t)y * W + std::min(W - 1, c + D / 2)) * 3 + k];
    hipError_t e = hipMemcpy(L, img.data(), img.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(R, img2.data(), img2.size(), hipMemcpyHostToDevice);
    // every copy reads the same pair and writes the same maps (identical values)
    const std::vector<BatchIO> io(copies, BatchIO{L, R, disp, valid});
    if (e == hipSuccess)
        e = hipMemcpy(tb.d_io, io.data(), io.size() * sizeof(BatchIO), hipMemcpyHostToDevice);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best_ms = 1e30f;
    *best = Tile{H, p.agg_iters == 2 ? std::min(2, D) : 1};
    for (const Tile& c : candidates(H, D, p.agg_iters)) {
        if (e != hipSuccess) break;
        for (BatchPair& pr : tb.pairs) {
            pr.band = c.band;
            pr.dchunk = c.dchunk;
        }
        if ((s = upload(&tb)) != DCO_OK) break;
        float ms[3];
        e = launch(&tb, st);  // warm-up
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = launch(&tb, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms[r], e0, e1);
        }
        if (e != hipSuccess) break;
        std::sort(ms, ms + 3);
        if (ms[1] < best_ms) {
            best_ms = ms[1];
            *best = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    release(&tb);
    if (e != hipSuccess) {
        dco_set_error("autotune of %dx%dx%d failed: %s", W, H, D, hipGetErrorString(e));
        return DCO_ERR_HIP;
    }
    return s;
}

}  // namespace

extern "C" dco_status dco_batch_create(dco_batch** out, int n, const int* W, const int* H,
                                       const int* D, const dco_params* p, void* stream) {
    if (!out) {
        dco_set_error("dco_batch_create: out is NULL");
        return DCO_ERR_ARG;
    }
    *out = nullptr;
    DCO_TRY(need(W, "W"));
    DCO_TRY(need(H, "H"));
    DCO_TRY(need(D, "D"));
    if (n < 1 || n > 4096) {
        dco_set_error("dco_batch_create: need 1 <= n <= 4096 (got %d)", n);
        return DCO_ERR_ARG;
    }
    dco_params prm;
    if (p)
        prm = *p;
    else
        dco_default_params(&prm);
    DCO_TRY(check_params(prm));
    if (prm.vote_iters != 0) {
        dco_set_error("dco_batch_create: the batched matcher has no Eq. 4 vote (vote_iters must "
                      "be 0; use dco_vote_refine per pair)");
        return DCO_ERR_ARG;
    }
    for (int i = 0; i < n; ++i) DCO_TRY(check_shape(W[i], H[i], D[i], prm));
    hipStream_t st = (hipStream_t)stream;
    // tile choice per size class: cache, else measure
    hipDeviceProp_t prop;
    int dev = 0;
    DCO_HIP_CHECK(hipGetDevice(&dev));
    DCO_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    char arch[64];
    snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
        if (*c == ':') *c = '\0';
    const bool tune = !(getenv("DCO_AUTOTUNE") && strcmp(getenv("DCO_AUTOTUNE"), "0") == 0);
    std::map<std::string, Tile> cache = tune ? read_cache() : std::map<std::string, Tile>();
    bool dirty = false;
    std::vector<Tile> tiles(n);
    for (int i = 0; i < n; ++i) {
        const std::string key = class_key(W[i], H[i], D[i], prm.agg_iters, arch);
        if (!tune) {
            tiles[i] = Tile{H[i], prm.agg_iters == 2 ? std::min(2, D[i]) : 1};
            continue;
        }
        auto it = cache.find(key);
        if (it == cache.end()) {
            Tile t;
            DCO_TRY(tune_class(prm, W[i], H[i], D[i], st, &t));
            cache[key] = t;
            dirty = true;
            it = cache.find(key);
        }
        tiles[i] = it->second;
    }
    if (dirty) write_cache(cache);

    dco_batch* b = new (std::nothrow) dco_batch();
    if (!b) {
        dco_set_error("host allocation failed");
        return DCO_ERR_OOM;
    }
    auto fail = [&](dco_status s) {
        release(b);
        delete b;
        return s;
    };
    dco_status s = make_base(b, n, prm);
    if (s != DCO_OK) return fail(s);
    b->stream = st;
    b->tiles = tiles;
    for (int i = 0; i < n; ++i) {
        if ((s = alloc_pair(b, b->pairs[i], W[i], H[i], D[i])) != DCO_OK) return fail(s);
        b->pairs[i].band = std::min(tiles[i].band, H[i]);
        b->pairs[i].dchunk = std::min(tiles[i].dchunk, D[i]);
    }
    if ((s = upload(b)) != DCO_OK) return fail(s);
    if ((s = pinned_alloc((void**)&b->h_io, sizeof(BatchIO) * n)) != DCO_OK) return fail(s);
    std::memset(b->h_io, 0, sizeof(BatchIO) * n);
    hipError_t e = hipEventCreateWithFlags(&b->io_copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch(b, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        dco_set_error("graph capture of the batched launch failed: %s", hipGetErrorString(e));
        return fail(DCO_ERR_HIP);
    }
    *out = b;
    return DCO_OK;
}

extern "C" void dco_batch_destroy(dco_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    release(b);
    delete b;
}

extern "C" dco_status dco_batch_match(dco_batch* b, const uint8_t* const* L,
                                      const uint8_t* const* R, float* const* disp,
                                      uint8_t* const* valid) {
    DCO_TRY(need(b, "batch"));
    DCO_TRY(need(L, "L"));
    DCO_TRY(need(R, "R"));
    DCO_TRY(need(disp, "disp"));
    DCO_TRY(need(valid, "valid"));
    for (int i = 0; i < b->n; ++i)
        if (!L[i] || !R[i] || !disp[i] || !valid[i]) {
            dco_set_error("dco_batch_match: a pointer of pair %d is NULL", i);
            return DCO_ERR_ARG;
        }
    // the staging table may still feed the previous call's copy
    if (b->io_pending) DCO_HIP_CHECK(hipEventSynchronize(b->io_copied));
    for (int i = 0; i < b->n; ++i) b->h_io[i] = BatchIO{L[i], R[i], disp[i], valid[i]};
    DCO_HIP_CHECK(hipMemcpyAsync(b->d_io, b->h_io, sizeof(BatchIO) * b->n,
                                 hipMemcpyHostToDevice, b->stream));
    DCO_HIP_CHECK(hipEventRecord(b->io_copied, b->stream));
    b->io_pending = true;
    DCO_HIP_CHECK(hipGraphLaunch(b->exec, b->stream));
    return DCO_OK;
}

extern "C" dco_status dco_batch_tile(const dco_batch* b, int i, int* strip_w, int* band_h,
                                     int* d_chunk) {
    DCO_TRY(need(b, "batch"));
    if (i < 0 || i >= b->n) {
        dco_set_error("dco_batch_tile: pair %d out of range", i);
        return DCO_ERR_ARG;
    }
    if (strip_w) *strip_w = kStripOut;
    if (band_h) *band_h = b->pairs[i].band;
    if (d_chunk) *d_chunk = b->pairs[i].dchunk;
    return DCO_OK;
}
