// Gram of sampled rows on float64 MFMA: G_b = X_r'X_r / m and C_b = X_r'Y_r / m.
//
// These are the normal-equation statistics of the bootstrap samples T^k of
// Alg. 1 / Alg. 2; the bootstrap is a row gather inside the kernel, so no
// resampled copy of X is ever written.  The product dominates the paper's
// single-node profile (its matrix multiplication inside LASSO-ADMM, Sec. IV-A.1).
//
// Columns: the design X (p columns) followed, when the response has fewer than
// 32 columns (the LASSO's y), by the response itself ("augmented" columns), so
// one symmetric product yields G, C = X'y/m and the mean squares y'y/m.  Many
// response columns (VAR) get their own rectangular tiles instead.
//
// Work decomposition: 128x128 output tiles of the lower triangle (plus C
// tiles), dealt XCD by XCD so that the tiles of one batch entry share an L2.
// A tile streams the sampled rows in chunks of 16 through LDS; 4 waves each own
// a 64x64 quadrant as 4x4 MFMA 16x16x4 blocks.  Interior tiles (all columns
// design columns) copy each gathered row segment from memory straight into LDS,
// 16 bytes per lane, into two alternating buffers.  Tiles that reach past the
// last design column stage through registers: the next chunk's gathered values
// are loaded while the current chunk is multiplied, and the row indices two
// chunks ahead, so the index -> value dependency never stalls the MFMAs.
//
// Short launches: with S workgroup slots on the chip (CUs x resident workgroups
// per CU) and U < S tiles (the estimation products over the union's columns,
// for instance), most of the chip would idle.  The tiles are then split over
// their rows into f parts (f <= 4, f U <= S) that run side by side; each part
// stores its raw accumulators and k_gram_fixup adds the parts in part order, so
// the result does not depend on timing (it differs from an unsplit tile at
// rounding level only).
#include <map>
#include <mutex>

#include "common.hpp"

namespace uoi {

namespace {
constexpr int GT = 128;  // tile edge
constexpr int GK = 16;   // rows per LDS chunk
constexpr int AUG_MAX = 32;  // response columns folded into the symmetric product
}

struct GramArgs {
    int m;
    const int32_t *rows;
    const int32_t *mcount;
    int p, pa;        // design columns, augmented response columns (0..AUG_MAX-1)
    const double *X;
    int ldx;
    int pe;           // response columns handled by C tiles (0 when augmented)
    const double *Y;
    int ldy;
    double *G, *C, *ss;  // ss: mean squares of the augmented responses (nullable)
    int T, Tc;
    const int32_t *wt;   // per-row weights (multiplicities) at stride m, or null
    int div;             // divisor of the sums (0: the row count)
    int tiles;           // tiles per batch entry
    int nfull;           // units 0..nfull-1 are whole tiles (batch-entry major)
    int fsplit;          // parts of each later tile (1: none split)
    double *part;        // raw partial tiles of the split units [unit - nfull][GT * GT]
    int direct;          // rows of X are 16-byte aligned (X and ldx even): interior tiles load rows into LDS directly
};

// tile index within a batch entry -> tile coordinates (lower triangle, then C tiles)
__device__ __forceinline__ void tile_coords(const GramArgs &g, int tile, int &ti, int &tj, bool &isC) {
    const int ntri = g.T * (g.T + 1) / 2;
    if (tile < ntri) {
        // row-major over the lower triangle, tj <= ti
        ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        while (ti * (ti + 1) / 2 > tile) --ti;
        tj = tile - ti * (ti + 1) / 2;
        isC = false;
    } else {
        tile -= ntri;
        ti = tile / g.Tc;
        tj = tile % g.Tc;
        isC = true;
    }
}

// Store product entry (i, j) of batch entry b, already divided by the row count.
__device__ __forceinline__ void gram_store(const GramArgs &g, int b, int i, int j, bool isC, double v) {
    const size_t gb = (size_t)b * g.p;
    const int naug = g.p + g.pa;
    if (isC) {
        if (i < g.p && j < g.pe) g.C[(gb + i) * g.pe + j] = v;
    } else if (j <= i && i < naug) {
        if (i < g.p) {                                   // design block, both halves
            g.G[(gb + i) * g.p + j] = v;
            if (j < i) g.G[(gb + j) * g.p + i] = v;
        }
        else if (j < g.p) g.C[(gb + j) * g.pa + (i - g.p)] = v;  // X'y block
        else if (i == j && g.ss) g.ss[(size_t)b * g.pa + (i - g.p)] = v;  // y'y diagonal
    }
}

// value of augmented column j of sampled row r
__device__ __forceinline__ double aug_col(const GramArgs &g, size_t r, int j) {
    if (j < g.p) return g.X[r * g.ldx + j];
    if (j < g.p + g.pa) return g.Y[r * g.ldy + (j - g.p)];
    return 0.0;
}

// A unit of work: one tile (or one part of a split tile) of batch entry b.
struct GramUnit {
    int b, i0, j0, mb, su, c0, c1;  // rows of chunks [c0, c1) of GK rows
    bool isC;
};

// The accumulators of a wave (a 64x64 quadrant) after the unit's rows: stored
// divided by the row count, or as raw parts of a split tile.
__device__ __forceinline__ void gram_finish(const GramArgs &g, const GramUnit &t, const dx4 (&acc)[4][4]) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1, lr = lane & 15, lk = lane >> 4;
    if (t.su >= 0) {  // a part of a split tile: raw accumulators, in register order
        double *P = g.part + (size_t)t.su * GT * GT;
#pragma unroll
        for (int fm = 0; fm < 4; ++fm)
#pragma unroll
            for (int fn = 0; fn < 4; ++fn)
#pragma unroll
                for (int e = 0; e < 4; ++e) P[((((wid * 4 + fm) * 4 + fn) * 4 + e) << 6) + lane] = acc[fm][fn][e];
        return;
    }
    const double inv = 1.0 / (double)(g.div > 0 ? g.div : t.mb);
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                gram_store(g, t.b, t.i0 + wm * 64 + fm * 16 + mfma_row(0.0, lk, e), t.j0 + wn * 64 + fn * 16 + lr,
                           t.isC, acc[fm][fn][e] * inv);
}

// One chunk of GK staged rows: acc += A_chunk' B_chunk, the A rows scaled by
// wrow (per staged row, from LDS) when W.
template <bool W>
__device__ __forceinline__ void gram_mma(const double (*As)[GT], const double (*Bs)[GT], const double *wrow,
                                         dx4 (&acc)[4][4]) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1, lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int s = 0; s < GK / 4; ++s) {
        double av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = As[4 * s + lk][wm * 64 + 16 * a + lr];
#pragma unroll
        for (int a = 0; a < 4; ++a) bv[a] = Bs[4 * s + lk][wn * 64 + 16 * a + lr];
        if (W) {
            const double ws = wrow[4 * s + lk];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] *= ws;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = mfma16x16x4(av[a], bv[q], acc[a][q]);
    }
}

// Interior tiles (every column of both sides a design column, rows of X 16-byte
// aligned): rows go from memory straight into LDS (16 bytes per lane, a wave
// fills one 128-column row of one side per instruction), two LDS buffers, one
// barrier per chunk.  Wave w stages rows 4w .. 4w+3 of each chunk; their indices
// and multipliers are loaded a chunk ahead by lanes 0-3 and taken into scalar
// registers, so a row's address is scalar arithmetic plus the lane's fixed
// 16-byte column offset.  The multiplier (weight, or 1; 0 for rows past the
// sample, which read row 0) scales the A values as they are read from LDS.
template <bool WGT>
__device__ __forceinline__ void gram_tile_direct(const GramArgs &g, const GramUnit &t, double (*As)[GK][GT],
                                                 double (*Bs)[GK][GT], double (*Ws)[GK]) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(tid >> 6));
    const int32_t *rb = g.rows + (size_t)t.b * g.m;
    const int32_t *wb = WGT ? g.wt + (size_t)t.b * g.m : nullptr;
    const int mb = t.mb;
    const double *xa = g.X + t.i0 + 2 * lane, *xb = g.X + t.j0 + 2 * lane;
    dx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = dx4{0, 0, 0, 0};
    // lanes 0-3 (and copies in the other lanes): index and multiplier of row
    // 4w + (lane & 3) of chunk c
    auto load_rows = [&](int c, int &vi, int &vw) {
        const int k = c * GK + 4 * w + (lane & 3);
        const int kc = k < mb ? k : 0;
        vi = rb[kc];
        const int wk = WGT ? wb[kc] : 1;  // loaded unconditionally (no branch around a load)
        vw = k < mb ? wk : 0;
    };
    // rows of chunk c (indices vi, multipliers vw) into buffer buf
    auto stage = [&](int buf, int vi, int vw) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const size_t row = (size_t)__builtin_amdgcn_readlane(vi, r) * g.ldx;
            __builtin_amdgcn_global_load_lds((const void *)(xa + row),
                                             (__attribute__((address_space(3))) void *)&As[buf][4 * w + r][0], 16, 0,
                                             0);
            __builtin_amdgcn_global_load_lds((const void *)(xb + row),
                                             (__attribute__((address_space(3))) void *)&Bs[buf][4 * w + r][0], 16, 0,
                                             0);
        }
        if (lane < 4) Ws[buf][4 * w + lane] = (double)vw;
    };
    int vi, vw, ni, nw;
    load_rows(t.c0, vi, vw);
    stage(t.c0 & 1, vi, vw);
    load_rows(t.c0 + 1, ni, nw);
    for (int c = t.c0; c < t.c1; ++c) {
        const int buf = c & 1;
        // this wave's copies into buffer buf (and every earlier load) complete,
        // then every wave's: the barrier also ends all reads of buffer buf ^ 1
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (c + 1 < t.c1) {
            stage(buf ^ 1, ni, nw);
            load_rows(c + 2, ni, nw);
        }
        gram_mma<true>(As[buf], Bs[buf], Ws[buf], acc);
    }
    gram_finish(g, t, acc);
}

// Other tiles: each thread stages one column of 8 rows per chunk through
// registers, the values of the next chunk in flight while the current one is
// multiplied.
template <bool WGT>
__device__ __forceinline__ void gram_tile_staged(const GramArgs &g, const GramUnit &t, double (*As)[GT],
                                                 double (*Bs)[GT]) {
    const int b = t.b, i0 = t.i0, j0 = t.j0, mb = t.mb;
    const bool isC = t.isC;
    const int32_t *rb = g.rows + (size_t)b * g.m;
    const int naug = g.p + g.pa;
    const int tid = threadIdx.x;
    // this thread stages rows kk = (tid >> 7) + 2q, column cc = tid & 127
    const int kk0 = tid >> 7, cc = tid & 127;
    const int ia = i0 + cc, jb = j0 + cc;

    dx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = dx4{0, 0, 0, 0};

    // Column sources of this thread's staged values are fixed for the kernel: a
    // valid base pointer and stride per side, and a 0/1 factor for columns past
    // the augmented width.  Loads are then issued without branches (rows past the
    // sample read row 0 and are zeroed), so a chunk's loads are all in flight
    // together instead of one at a time.
    const double *pa = g.X, *pb = g.X;
    int lda = g.ldx, ldb = g.ldx;
    double am = 0.0, bm = 0.0;
    if (ia < g.p) { pa = g.X + ia; am = 1.0; }
    else if (ia < naug) { pa = g.Y + (ia - g.p); lda = g.ldy; am = 1.0; }
    if (isC) {
        if (jb < g.pe) { pb = g.Y + jb; ldb = g.ldy; bm = 1.0; }
    } else if (jb < g.p) { pb = g.X + jb; bm = 1.0; }
    else if (jb < naug) { pb = g.Y + (jb - g.p); ldb = g.ldy; bm = 1.0; }
    const int32_t *wb = WGT ? g.wt + (size_t)b * g.m : nullptr;
    // Row indices and weights of a chunk are requested two chunks ahead and kept
    // as loaded (the validity test and the conversion happen at their use), so no
    // wait is needed until then.
    int idx1[8], idx2[8], wi1[8], wi2[8];
    double ra[8], rbv[8];
    auto load_idx = [&](int k0, int (&idx)[8], int (&wi)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = k0 + kk0 + 2 * q;
            const int kc = k < mb ? k : 0;
            idx[q] = rb[kc];
            if (WGT) wi[q] = wb[kc];
        }
    };
    // values of the chunk starting at row k0 (rows past the sample are zeroed)
    auto load_val = [&](int k0, const int (&idx)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool ok = k0 + kk0 + 2 * q < mb;
            const size_t r = (size_t)idx[q];
            ra[q] = pa[r * lda] * (ok ? am : 0.0);
            rbv[q] = pb[r * ldb] * (ok ? bm : 0.0);
        }
    };
    auto store = [&](const int (&wi)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // the weight (multiplicity) on one side
            As[kk0 + 2 * q][cc] = WGT ? ra[q] * (double)wi[q] : ra[q];
            Bs[kk0 + 2 * q][cc] = rbv[q];
        }
    };

    // this unit's chunks of GK rows: [c0, c1)
    const int c0 = t.c0, c1 = t.c1;
    load_idx(c0 * GK, idx1, wi1);
    load_val(c0 * GK, idx1);
    store(wi1);
    load_idx((c0 + 1) * GK, idx1, wi1);
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
        const bool more = c + 1 < c1;
        if (more) {
            load_val((c + 1) * GK, idx1);        // values of chunk c+1
            load_idx((c + 2) * GK, idx2, wi2);   // indices and weights of chunk c+2
        }
        gram_mma<false>(As, Bs, nullptr, acc);
        __syncthreads();
        if (more) {
            store(wi1);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                idx1[q] = idx2[q];
                wi1[q] = wi2[q];
            }
        }
        __syncthreads();
    }

    gram_finish(g, t, acc);
}

// ROLE only names the instance (0: selection products of the bootstrap samples,
// 1: estimation products), so kernel profiles keep the two apart.
template <int ROLE, bool WGT>
__global__ __launch_bounds__(256, 2) void k_gram_f64(GramArgs g) {
    __shared__ double As[2][GK][GT];
    __shared__ double Bs[2][GK][GT];
    __shared__ double Ws[2][GK];
    // unit -> (tile of batch entry b, part q of f).  Units are dealt so that each
    // XCD takes a contiguous range: the tiles of one batch entry then share that
    // XCD's L2 while they stream the same rows (34 % less fetched from memory at
    // the benchmark, 3 % faster).
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    const int su = u - g.nfull;                      // index among split units, or < 0
    const int f = su < 0 ? 1 : g.fsplit;
    const int q = su < 0 ? 0 : su % f;
    const int lt = su < 0 ? u : g.nfull + su / f;
    GramUnit t;
    t.b = lt / g.tiles;
    t.su = su;
    int ti, tj;
    tile_coords(g, lt % g.tiles, ti, tj, t.isC);
    t.i0 = ti * GT;
    t.j0 = tj * GT;
    t.mb = g.mcount ? g.mcount[t.b] : g.m;
    const int nchunk = (t.mb + GK - 1) / GK;
    t.c0 = (int)((int64_t)q * nchunk / f);
    t.c1 = (int)((int64_t)(q + 1) * nchunk / f);
    const bool direct = g.direct && !t.isC && t.i0 + GT <= g.p && t.j0 + GT <= g.p;
    if (direct)
        gram_tile_direct<WGT>(g, t, As, Bs, Ws);
    else
        gram_tile_staged<WGT>(g, t, As[0], Bs[0]);
}

// Split tiles: the sum of their parts in part order, divided by the row count.
// One workgroup per split tile, threads laid out as in k_gram_f64.
__global__ __launch_bounds__(256) void k_gram_fixup(GramArgs g) {
    const int lt = g.nfull + blockIdx.x;
    const int b = lt / g.tiles;
    int ti, tj;
    bool isC;
    tile_coords(g, lt % g.tiles, ti, tj, isC);
    const int i0 = ti * GT, j0 = tj * GT;
    const int mb = g.mcount ? g.mcount[b] : g.m;
    const double inv = 1.0 / (double)(g.div > 0 ? g.div : mb);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1, lr = lane & 15, lk = lane >> 4;
    const double *P = g.part + (size_t)blockIdx.x * g.fsplit * GT * GT;
    for (int r = 0; r < 64; ++r) {  // r = (fm, fn, t)
        const int fm = r >> 4, fn = (r >> 2) & 3, t = r & 3;
        const size_t o = ((size_t)(wid * 64 + r) << 6) + lane;
        double v = P[o];
        for (int h = 1; h < g.fsplit; ++h) v += P[(size_t)h * GT * GT + o];
        gram_store(g, b, i0 + wm * 64 + fm * 16 + mfma_row(0.0, lk, t), j0 + wn * 64 + fn * 16 + lr, isC, v * inv);
    }
}

// Upper triangle from the lower one: G[j][i] = G[i][j] for i > j, by 32x32
// tiles transposed through LDS (coalesced reads and writes).
__global__ void k_symmetrize(int p, double *__restrict__ G) {
    __shared__ double t[32][33];
    const int b = blockIdx.z;
    const int bi = blockIdx.y, bj = blockIdx.x;  // source tile rows bi, columns bj, bi >= bj
    if (bj > bi) return;
    double *Gb = G + (size_t)b * p * p;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int r = ty; r < 32; r += 8) {
        int i = bi * 32 + r, j = bj * 32 + tx;
        if (i < p && j < p) t[r][tx] = Gb[(size_t)i * p + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int i = bj * 32 + r, j = bi * 32 + tx;  // destination (i, j) = source (j, i)
        if (i < p && j < p && j > i) Gb[(size_t)i * p + j] = t[tx][r];
    }
}

// ss[b][e] = sum over sampled rows of Y[r][e]^2 / m
__global__ __launch_bounds__(256) void k_colsq(int m, const int32_t *__restrict__ rows,
                                               const int32_t *__restrict__ mcount, int pe,
                                               const double *__restrict__ Y, int ldy,
                                               double *__restrict__ ss) {
    __shared__ double part[4][64];
    int b = blockIdx.y;
    int e = blockIdx.x * 64 + (threadIdx.x & 63);
    int ph = threadIdx.x >> 6;
    int mb = mcount ? mcount[b] : m;
    const int32_t *rb = rows + (size_t)b * m;
    double acc = 0.0;
    if (e < pe)
        for (int k = ph; k < mb; k += 4) {
            double v = Y[(size_t)rb[k] * ldy + e];
            acc += v * v;
        }
    part[ph][threadIdx.x & 63] = acc;
    __syncthreads();
    if (ph == 0 && e < pe) {
        double s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                   part[3][threadIdx.x];
        ss[(size_t)b * pe + e] = s / (double)mb;
    }
}

namespace {
// Workgroup slots of a Gram instance on the current device: CUs x workgroups of
// that instance resident per CU.
template <int ROLE, bool WGT>
int gram_slots() {
    static std::mutex mu;
    static std::map<int, int> cache;
    int dev = 0;
    UOI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0, per = 0;
    UOI_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    UOI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(&k_gram_f64<ROLE, WGT>),
                                                         256, 0));
    const int slots = std::max(1, cus * std::max(per, 1));
    cache[dev] = slots;
    return slots;
}

int gram_slots_of(int role, bool weighted) {
    if (weighted) return gram_slots<0, true>();
    return role == 0 ? gram_slots<0, false>() : gram_slots<1, false>();
}

// Tile counts of a product (see GramArgs) and the split of its last partial round.
struct GramPlan {
    int T, Tc, pa, pe, tiles, nfull, f, units;
    size_t part_bytes;
};

GramPlan gram_plan(int nb, int m, int p, int pe, bool have_c, int slots) {
    GramPlan pl{};
    const bool aug = have_c && pe > 0 && pe < AUG_MAX;
    pl.pa = aug ? pe : 0;
    pl.pe = (have_c && !aug) ? pe : 0;
    pl.T = (int)cdiv(p + pl.pa, GT);
    pl.Tc = pl.pe > 0 ? (int)cdiv(pl.pe, GT) : 0;
    pl.tiles = pl.T * (pl.T + 1) / 2 + (int)cdiv(p, GT) * pl.Tc;
    const int64_t total = (int64_t)nb * pl.tiles;
    // Only a launch shorter than one round is split: after full rounds the last
    // round's workgroups run alone on their compute units, faster than in a full
    // round, and the fixup pass costs more than the split saves.
    const int rem = total < slots ? (int)total : 0;
    int f = rem ? std::min(4, slots / rem) : 1;
    f = std::min<int64_t>(f, std::max<int64_t>(1, cdiv(m, GK) / 4));  // at least 4 chunks per part
    if (f < 2) {
        pl.f = 1;
        pl.nfull = (int)total;
        pl.units = (int)total;
        pl.part_bytes = 0;
    } else {
        pl.f = f;
        pl.nfull = (int)(total - rem);
        pl.units = pl.nfull + rem * f;
        pl.part_bytes = sizeof(double) * (size_t)rem * f * GT * GT;
    }
    return pl;
}

// Launch a product planned by gram_plan; without room for the partial tiles no
// tile is split.
void run_gram(hipStream_t s, GramArgs g, GramPlan pl, int role, bool weighted, void *part, size_t part_bytes) {
    if (pl.f > 1 && (part == nullptr || part_bytes < pl.part_bytes)) {
        const int rem = (pl.units - pl.nfull) / pl.f;
        pl.f = 1;
        pl.nfull = pl.units = pl.nfull + rem;
    }
    g.pa = pl.pa;
    g.pe = pl.pe;
    g.T = pl.T;
    g.Tc = pl.Tc;
    g.tiles = pl.tiles;
    g.nfull = pl.nfull;
    g.fsplit = pl.f;
    g.part = (double *)part;
    if (pl.units == 0) return;
    if (weighted)
        hipLaunchKernelGGL((k_gram_f64<0, true>), dim3(pl.units), dim3(256), 0, s, g);
    else if (role == 0)
        hipLaunchKernelGGL((k_gram_f64<0, false>), dim3(pl.units), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gram_f64<1, false>), dim3(pl.units), dim3(256), 0, s, g);
    UOI_LAUNCH_CHECK();
    if (pl.f > 1) {
        hipLaunchKernelGGL(k_gram_fixup, dim3((pl.units - pl.nfull) / pl.f), dim3(256), 0, s, g);
        UOI_LAUNCH_CHECK();
    }
}
}  // namespace

size_t gram_part_bytes(int nb, int m, int p, int pe, bool have_c, int role, bool weighted) {
    return gram_plan(nb, m, p, pe, have_c, gram_slots_of(role, weighted)).part_bytes;
}

void launch_gram_f64(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *mcount,
                     int p, const double *X, int ldx, int pe, const double *Y, int ldy,
                     double *G, double *C, double *ss, int role, void *part, size_t part_bytes) {
    GramArgs g{};
    g.m = m; g.rows = rows; g.mcount = mcount; g.p = p; g.X = X; g.ldx = ldx;
    g.Y = Y; g.ldy = ldy; g.G = G; g.C = C; g.ss = ss;
    g.direct = ldx % 2 == 0 && ((uintptr_t)X & 15) == 0;
    const GramPlan pl = gram_plan(nb, m, p, pe, C != nullptr, gram_slots_of(role, false));
    run_gram(s, g, pl, role, false, part, part_bytes);
}

void launch_gram_f64_weighted(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *w,
                              const int32_t *mcount, int div, int p, const double *X, int ldx, int pe,
                              const double *Y, int ldy, double *G, double *C, double *ss, void *part,
                              size_t part_bytes) {
    GramArgs g{};
    g.m = m; g.rows = rows; g.mcount = mcount; g.p = p; g.X = X; g.ldx = ldx;
    g.Y = Y; g.ldy = ldy; g.G = G; g.C = C; g.ss = ss; g.wt = w; g.div = div;
    g.direct = ldx % 2 == 0 && ((uintptr_t)X & 15) == 0;
    const GramPlan pl = gram_plan(nb, m, p, pe, C != nullptr, gram_slots_of(0, true));
    run_gram(s, g, pl, 0, true, part, part_bytes);
}

void launch_symmetrize(hipStream_t s, int nb, int p, double *G) {
    const int T32 = (int)cdiv(p, 32);
    hipLaunchKernelGGL(k_symmetrize, dim3(T32, T32, nb), dim3(32, 8), 0, s, p, G);
    UOI_LAUNCH_CHECK();
}

void launch_colsq(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *mcount,
                  int pe, const double *Y, int ldy, double *ss) {
    hipLaunchKernelGGL(k_colsq, dim3(cdiv(pe, 64), nb), dim3(256), 0, s, m, rows, mcount, pe, Y,
                       ldy, ss);
    UOI_LAUNCH_CHECK();
}

// --------------------------------------------------------------------------
// Full-data sums split over contiguous row slices (one Gram launch with a
// slice per batch entry keeps the chip busy when only one product is needed),
// and training statistics as their complement to the evaluation statistics.

// Slice k holds rows k*mp .. min((k+1)*mp, n) - 1.
__global__ void k_row_slices(int n, int mp, int32_t *__restrict__ rows, int32_t *__restrict__ cnt) {
    const int k = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = max(0, min(mp, n - k * mp));
    if (r == 0) cnt[k] = c;
    if (r < c) rows[(size_t)k * mp + r] = k * mp + r;
}

// S[i] = sum_k cnt_k P[k][i]  (un-normalised sums of the slices)
__global__ void k_sum_slices(size_t len, int ns, const double *__restrict__ P,
                             const int32_t *__restrict__ cnt, double *__restrict__ S) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (size_t)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int k = 0; k < ns; ++k) a += (double)cnt[k] * P[(size_t)k * len + i];
        S[i] = a;
    }
}

// T[b][i] = (S[i] - ne_b E[b][i]) / nt_b
__global__ void k_complement(size_t len, const double *__restrict__ S, const double *__restrict__ E,
                             int nt_c, int ne_c, const int32_t *__restrict__ nt,
                             const int32_t *__restrict__ ne, double *__restrict__ T) {
    const int b = blockIdx.y;
    const double fe = ne ? (double)ne[b] : (double)ne_c;
    const double inv = 1.0 / (nt ? (double)nt[b] : (double)nt_c);
    const double *Eb = E + (size_t)b * len;
    double *Tb = T + (size_t)b * len;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (size_t)gridDim.x * blockDim.x)
        Tb[i] = (S[i] - fe * Eb[i]) * inv;
}

namespace {
struct SliceShape {
    int ns, mp;
};
SliceShape slice_shape(int n, int p, int pe) {
    const bool aug = pe > 0 && pe < AUG_MAX;
    const int T = (int)cdiv(p + (aug ? pe : 0), GT);
    const int Tc = aug || pe == 0 ? 0 : (int)cdiv(pe, GT);
    const int tiles = T * (T + 1) / 2 + (int)cdiv(p, GT) * Tc;
    int ns = (int)std::min<int64_t>(32, cdiv(768, tiles));
    ns = std::max(1, std::min(ns, n / 64));
    const int mp = (int)cdiv(n, ns);
    return {(int)cdiv(n, mp), mp};
}
}  // namespace

// enough for any design width up to p (a caller may run on a column subset)
size_t complement_work_bytes(int n, int p, int pe) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t most = 0;
    for (int pp = 1; pp <= p; ++pp) {
        const SliceShape sh = slice_shape(n, pp, pe);
        most = std::max(most, al(sizeof(int32_t) * (size_t)sh.ns * sh.mp) + al(sizeof(int32_t) * sh.ns) +
                                  al(sizeof(double) * (size_t)sh.ns * pp * (pp + pe)) +
                                  al(sizeof(double) * (size_t)pp * (pp + pe)) +
                                  al(gram_part_bytes(sh.ns, sh.mp, pp, pe, true, 1, false)));
    }
    return most;
}

void launch_train_from_eval(hipStream_t s, int nb, int n, int p, const double *X, int ldx, int pe,
                            const double *Y, int ldy, const double *GE, const double *CE,
                            int nt_c, int ne_c, const int32_t *nt, const int32_t *ne, double *GT,
                            double *CT, void *work) {
    const SliceShape sh = slice_shape(n, p, pe);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *w = (char *)work;
    int32_t *rows = (int32_t *)w;
    w += al(sizeof(int32_t) * (size_t)sh.ns * sh.mp);
    int32_t *cnt = (int32_t *)w;
    w += al(sizeof(int32_t) * sh.ns);
    double *Gp = (double *)w;
    double *Cp = Gp + (size_t)sh.ns * p * p;
    w += al(sizeof(double) * (size_t)sh.ns * p * (p + pe));
    double *SG = (double *)w;
    double *SC = SG + (size_t)p * p;
    w += al(sizeof(double) * (size_t)p * (p + pe));
    const size_t pb = gram_part_bytes(sh.ns, sh.mp, p, pe, true, 1, false);

    hipLaunchKernelGGL(k_row_slices, dim3(cdiv(sh.mp, 256), sh.ns), dim3(256), 0, s, n, sh.mp, rows, cnt);
    UOI_LAUNCH_CHECK();
    launch_gram_f64(s, sh.ns, sh.mp, rows, cnt, p, X, ldx, pe, Y, ldy, Gp, Cp, nullptr, 1, w, pb);
    const size_t lg = (size_t)p * p, lc = (size_t)p * pe;
    const int nbk = 1024;
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)std::min<size_t>(cdiv(lg, 256), nbk)), dim3(256), 0,
                       s, lg, sh.ns, Gp, cnt, SG);
    UOI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)std::min<size_t>(cdiv(lc, 256), nbk)), dim3(256), 0,
                       s, lc, sh.ns, Cp, cnt, SC);
    UOI_LAUNCH_CHECK();
    const int gx = (int)std::min<size_t>(cdiv(lg, 256), 128);
    hipLaunchKernelGGL(k_complement, dim3(gx, nb), dim3(256), 0, s, lg, SG, GE, nt_c, ne_c, nt, ne, GT);
    UOI_LAUNCH_CHECK();
    const int gc = (int)std::min<size_t>(cdiv(lc, 256), 128);
    hipLaunchKernelGGL(k_complement, dim3(gc, nb), dim3(256), 0, s, lc, SC, CE, nt_c, ne_c, nt, ne, CT);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
