// Batched Q-less TSQR: many independent tall-skinny matrices of uneven m and
// n in one persistent stage-1 launch plus one launch per tree level (paper
// Alg. 2 applied per matrix).
//
// The host plan cuts every matrix into row tiles (about tile_bytes each),
// orders all tiles longest first and lists the tree groups of every level.
// Stage 1: a fixed grid of wavefronts takes the tiles in turn (wavefront w
// takes tiles w, w + W, w + 2W, ...); each folds its tile into an R with the
// same per-n code as qless_tsqr_r and writes it to the matrix's level-0 slot
// (a matrix of one tile writes its final R at once).  Tree level l: the
// groups of fan_in stacked triangles of every matrix that still has more
// than one are folded by the same grid, level l+1 slots or, for a root, the
// matrix's sign-normalised R.  Wavefronts never wait for one another, and no
// state survives a launch, so a captured graph of the sequence replays
// as is.  Optionally the previous contents of a matrix's R are stacked into
// its root (R([R_old; X])), which is how a caller keeps a running R over
// chunks of rows.
#include <algorithm>
#include <array>
#include <new>
#include <vector>

#include "batched_kernels.h"

struct qless_batch_plan {
    std::vector<qless::BatchMat> mats;
    std::vector<int2> tiles;                  // (matrix, tile): by width class, longest first within a class
    std::vector<qless::BatchGroup> groups;    // tree groups, by level, then by width class
    int64_t tile_end[qless::batch_detail::kBatchClasses] = {};          // class c: tiles [end[c-1], end[c])
    std::vector<std::array<int64_t, qless::batch_detail::kBatchClasses>> level_end;   // per level and class
    int np_max[qless::batch_detail::kBatchClasses] = {};
    int64_t slot_doubles = 0;
    size_t off_tiles = 0, off_groups = 0, off_slots = 0, bytes = 0;
    int waves_cap = 0;
};

namespace qless {
namespace {

using batch_detail::kBatchWpb;
using batch_detail::kFanIn;

// Padded width of the batched kernels for n (the widths of QLESS_BATCH_SWITCH).
int batch_np(int64_t n) {
    static const int widths[] = {1, 2, 4, 8, 16, 24, 32, 40, 48, 56, 64};
    for (int w : widths)
        if (n <= w) return w;
    return 64;
}

// Panel rows of the instance of a padded width (tiles are whole panels).
int64_t batch_panel_rows(int np) {
    using batch_detail::batch_rpl;
    using tsqr_detail::panel_rows;
    switch (np) {
        case 1: return panel_rows<1, batch_rpl(1)>();
        case 2: return panel_rows<2, batch_rpl(2)>();
        case 4: return panel_rows<4, batch_rpl(4)>();
        case 8: return panel_rows<8, batch_rpl(8)>();
        case 16: return panel_rows<16, batch_rpl(16)>();
        case 24: return panel_rows<24, batch_rpl(24)>();
        case 32: return panel_rows<32, batch_rpl(32)>();
        case 40: return panel_rows<40, batch_rpl(40)>();
        case 48: return panel_rows<48, batch_rpl(48)>();
        case 56: return panel_rows<56, batch_rpl(56)>();
        default: return panel_rows<64, batch_rpl(64)>();
    }
}

}  // namespace

hipError_t launch_batched_stage(int cls, const BatchMat* mats, const int2* tiles, int64_t ntiles, int64_t nwaves,
                                double* slots, int r_doubles, bool staged, hipStream_t s);
hipError_t launch_batched_tree(int cls, const BatchMat* mats, const BatchGroup* groups, int64_t ngroups,
                               int64_t nwaves, double* slots, int r_doubles, hipStream_t s);

// Tree fan-in of a matrix of n columns: the single-matrix plan's (one panel
// of stacked triangles per wavefront for n <= 16, else 4, or the autotuner's
// choice), within [2, 64].
int batch_fan_in(int64_t n) {
    int fan = 0;
    if (tsqr_tune_get(n, nullptr, &fan, nullptr) != QLESS_OK || fan < 2) fan = kFanIn;
    return std::min(fan, 64);
}

int batch_plan_create(const qless_matrix_desc* d, int32_t count, int64_t tile_bytes, int waves_per_cu,
                      qless_batch_plan** out) {
    using batch_detail::batch_class;
    using batch_detail::kBatchClasses;
    if (out == nullptr || d == nullptr || count < 1) return QLESS_ERR_ARG;
    *out = nullptr;
    if (tile_bytes <= 0) tile_bytes = 4 << 20;
    if (waves_per_cu <= 0) waves_per_cu = 8;
    for (int32_t i = 0; i < count; ++i) {
        if (d[i].n < 1 || d[i].m < 0) return QLESS_ERR_ARG;
        if (d[i].n > QLESS_MAX_N) return QLESS_ERR_UNSUPPORTED;
        if (d[i].R == nullptr || d[i].ldr < d[i].n) return QLESS_ERR_ARG;
        if (d[i].m > 0 && (d[i].X == nullptr || d[i].ldx < d[i].n)) return QLESS_ERR_ARG;
    }
    qless_batch_plan* p = new (std::nothrow) qless_batch_plan;
    if (!p) return QLESS_ERR_ARG;
    int64_t slots = 0;
    // (class, rows * n, (matrix, tile)) for the tile order
    std::vector<std::pair<std::pair<int, int64_t>, int2>> order;
    // levels[l][c]: groups of tree level l + 1 in width class c
    std::vector<std::array<std::vector<BatchGroup>, kBatchClasses>> levels;
    for (int32_t i = 0; i < count; ++i) {
        BatchMat M{};
        M.X = d[i].X;
        M.R = d[i].R;
        M.m = d[i].m;
        M.ldx = d[i].m > 0 ? d[i].ldx : d[i].n;
        M.ldr = d[i].ldr;
        M.n = (int)d[i].n;
        M.np = batch_np(d[i].n);
        M.accumulate = d[i].accumulate ? 1 : 0;
        const int cls = batch_class(M.np);
        const int fan = batch_fan_in(d[i].n);
        const int64_t panel = batch_panel_rows(M.np);
        int64_t tr = tile_bytes / (8 * d[i].n);
        tr = std::max<int64_t>(panel, tr / panel * panel);
        M.tile_rows = tr;
        M.ntiles = (int)std::max<int64_t>(1, ceil_div(d[i].m, tr));
        M.slot_base = slots;
        // slots of level l hold the c_l triangles of that level (c_0 = ntiles);
        // the root (c_l = 1) is written to R instead
        const int64_t nn = d[i].n * d[i].n;
        int64_t base = slots, c = M.ntiles;
        if (c > 1) slots += c * nn;
        for (int l = 1; c > 1; ++l) {
            const int64_t cn = ceil_div(c, fan);
            const int64_t next_base = slots;
            if (cn > 1) slots += cn * nn;
            if ((int)levels.size() < l) levels.resize(l);
            for (int64_t g = 0; g < cn; ++g) {
                BatchGroup G;
                G.src = base + g * fan * nn;
                G.dst = cn == 1 ? -1 : next_base + g * nn;
                G.mat = i;
                G.gsize = (int)std::min<int64_t>(fan, c - g * fan);
                levels[l - 1][cls].push_back(G);
            }
            base = next_base;
            c = cn;
        }
        p->np_max[cls] = std::max(p->np_max[cls], M.np);
        p->mats.push_back(M);
        for (int t = 0; t < M.ntiles; ++t) {
            const int64_t rows = std::min<int64_t>(tr, std::max<int64_t>(0, d[i].m - (int64_t)t * tr));
            order.push_back({{cls, rows * d[i].n}, make_int2(i, t)});
        }
    }
    std::stable_sort(order.begin(), order.end(), [](const auto& a, const auto& b) {
        return a.first.first != b.first.first ? a.first.first < b.first.first : a.first.second > b.first.second;
    });
    p->tiles.reserve(order.size());
    for (auto& o : order) {
        p->tiles.push_back(o.second);
        p->tile_end[o.first.first] = (int64_t)p->tiles.size();
    }
    for (int c = 1; c < kBatchClasses; ++c) p->tile_end[c] = std::max(p->tile_end[c], p->tile_end[c - 1]);
    for (auto& lv : levels) {
        std::array<int64_t, kBatchClasses> ends{};
        for (int c = 0; c < kBatchClasses; ++c) {
            p->groups.insert(p->groups.end(), lv[c].begin(), lv[c].end());
            ends[c] = (int64_t)p->groups.size();
        }
        p->level_end.push_back(ends);
    }
    p->slot_doubles = slots;
    p->off_tiles = align_up(p->mats.size() * sizeof(BatchMat), 256);
    p->off_groups = p->off_tiles + align_up(p->tiles.size() * sizeof(int2), 256);
    p->off_slots = p->off_groups + align_up(std::max<size_t>(p->groups.size(), 1) * sizeof(BatchGroup), 256);
    p->bytes = p->off_slots + align_up((size_t)std::max<int64_t>(slots, 1) * sizeof(double), 256);
    const DeviceInfo& di = current_device_info();
    p->waves_cap = di.num_cus * waves_per_cu;
    *out = p;
    return QLESS_OK;
}

int batch_plan_upload(const qless_batch_plan* p, void* work, size_t work_bytes, hipStream_t s) {
    if (p == nullptr) return QLESS_ERR_ARG;
    if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) || work_bytes < p->bytes)
        return QLESS_ERR_WORKSPACE;
    char* b = static_cast<char*>(work);
    hipError_t e = hipMemcpyAsync(b, p->mats.data(), p->mats.size() * sizeof(BatchMat), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b + p->off_tiles, p->tiles.data(), p->tiles.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !p->groups.empty())
        e = hipMemcpyAsync(b + p->off_groups, p->groups.data(), p->groups.size() * sizeof(BatchGroup),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the plan's host arrays may be reused right after
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int batch_run(const qless_batch_plan* p, void* work, size_t work_bytes, hipStream_t s) {
    using batch_detail::kBatchClasses;
    if (p == nullptr) return QLESS_ERR_ARG;
    if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) || work_bytes < p->bytes)
        return QLESS_ERR_WORKSPACE;
    char* b = static_cast<char*>(work);
    const BatchMat* mats = reinterpret_cast<const BatchMat*>(b);
    double* slots = reinterpret_cast<double*>(b + p->off_slots);
    const int2* tiles = reinterpret_cast<const int2*>(b + p->off_tiles);
    const BatchGroup* groups = reinterpret_cast<const BatchGroup*>(b + p->off_groups);
    auto region = [&](int c) { return p->np_max[c] * (p->np_max[c] + 1) / 2 + p->np_max[c]; };
    // stage 1: one persistent launch per width class present
    int64_t lo = 0;
    for (int c = 0; c < kBatchClasses; ++c) {
        const int64_t nt = p->tile_end[c] - lo;
        if (nt > 0 && launch_batched_stage(c, mats, tiles + lo, nt, std::min<int64_t>(nt, p->waves_cap), slots,
                                           region(c), c == 0, s) != hipSuccess)
            return QLESS_ERR_HIP;
        lo = p->tile_end[c];
    }
    // tree levels, each class's groups of a level in one launch
    int64_t g0 = 0;
    for (const auto& ends : p->level_end) {
        for (int c = 0; c < kBatchClasses; ++c) {
            const int64_t ng = ends[c] - g0;
            if (ng > 0 && launch_batched_tree(c, mats, groups + g0, ng, std::min<int64_t>(ng, p->waves_cap), slots,
                                              region(c), s) != hipSuccess)
                return QLESS_ERR_HIP;
            g0 = ends[c];
        }
    }
    return QLESS_OK;
}

void batch_plan_destroy(qless_batch_plan* p) { delete p; }
size_t batch_plan_bytes(const qless_batch_plan* p) { return p ? p->bytes : 0; }
int64_t batch_plan_tiles(const qless_batch_plan* p) { return p ? (int64_t)p->tiles.size() : 0; }

}  // namespace qless
