// Batched uneven CP and Kronecker sketches (Sections 3.1 and 4.3 of the
// paper) in persistent kernels, one per FFT size class, optionally replayed
// from a single captured hipGraph.
//
// Work decomposition.  Every computation of the batch is split into tiles:
// a CP sketch into (sketch d, slice q, rank chunk) forward tiles, a
// Kronecker sketch into one tile per sketch d.  Tiles of one FFT size P form
// a class; a class kernel runs a fixed number of workgroups that take tiles
// from a queue (one atomic counter) in decreasing order of estimated cost,
// so long tiles start first and short ones fill the tail.
//
// Completion.  A CP forward tile of several rank chunks writes its partial
// spectrum, releases it (device-scope fence) and counts itself on the
// counter of its slice (d, q); the workgroup that completes the count
// acquires the partials and inverts that slice (a single chunk inverts in
// place).  With several slices, each slice writes its term of y to a slice
// row and counts itself on the counter of sketch d; the last one sums the
// rows in slice order.  Counters and queue heads are reset by the kernels
// themselves (the last finisher), so a captured graph replays without any
// memset node.
//
// Count sketches.  CP tiles scatter each factor column into fixed-point LDS
// bins scaled to the column's maximum; one small kernel at the head of the
// run (and of the graph) computes the maxima of every CP item's columns,
// one wave per column.
#include "fcs_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

#include "cp_tile.h"

using namespace fcsfft;
using namespace fcscp;

namespace {

constexpr int NCLASS = 7;            // P = 2^8 .. 2^14

struct BatchTile {
    int32_t inst, d, q, chunk;
};

struct BatchArgs {
    const CpDesc *desc;
    const BatchTile *tiles;          // this class, costliest first
    int ntiles;
    int *head;                      // queue head of this class
    int *done;                      // workgroups of this class that left
    int *cnt;                       // per (computation, sketch) completion counters
};

// Queue tickets and the last-tile flag.  A workgroup of one wave (P <= 1024)
// has its barriers removed by the compiler, so it must not pass values from
// one lane to the others through LDS inside the persistent loop: a lane-0
// branch there may be moved out of the loop iteration the other lanes are
// in.  Such workgroups let every lane take part in the atomic (adding 1 from
// lane 0 and 0 from the others) and broadcast lane 0's result with
// readfirstlane, so every branch of the loop is wave-uniform.  Larger
// workgroups keep real barriers and broadcast through LDS.
template <int P>
__device__ __forceinline__ int wg_atomic_ticket(int *ctr, int *slot) {
    if constexpr (Shape<P>::T == 64) {
        const int v = atomicAdd(ctr, threadIdx.x == 0 ? 1 : 0);
        return __builtin_amdgcn_readfirstlane(v);
    } else {
        if (threadIdx.x == 0) *slot = atomicAdd(ctr, 1);
        __syncthreads();
        const int v = __builtin_amdgcn_readfirstlane(*slot);
        __syncthreads();
        return v;
    }
}

template <int P>
__device__ __forceinline__ void batch_tile(const BatchArgs &a, int t, float2 *lds, int *slot) {
    const BatchTile tl = a.tiles[t];
    const CpDesc &c = a.desc[tl.inst];
    const int kind = __builtin_amdgcn_readfirstlane(c.kind);
    const int d = __builtin_amdgcn_readfirstlane(tl.d);
    if (kind == FCS_DESC_KRON) {
        kron_sketch<P>(c, d, lds);
        return;
    }
    const int q = __builtin_amdgcn_readfirstlane(tl.q);
    const int chunk = __builtin_amdgcn_readfirstlane(tl.chunk);
    const int nch = __builtin_amdgcn_readfirstlane(c.nchunks);
    const int Qh = __builtin_amdgcn_readfirstlane(c.s.Qh);
    float2 acc[Shape<P>::E];
    // second-entry words on demand: persistent occupancy depends on registers
    cp_tile<P, false>(c, d, q, chunk, lds, acc);
    if (nch == 1) {
        finish_slice<P>(c, d, q, lds, acc, slice_dst(c, d, q), false);
    } else {
        // the last chunk of slice (d, q) to finish inverts the slice
        store_partial<P>(c, d, q, chunk, acc);
        int *cnt = a.cnt + c.cnt_slice + d * Qh + q;
        __threadfence();                 // release this tile's partial spectrum
        __syncthreads();
        if (wg_atomic_ticket<P>(cnt, slot) != nch - 1) return;
        __threadfence();                 // acquire the other chunks' partials
        slice_from_partials<P>(c, d, q, lds, nch);
        atomicExch(cnt, 0);              // ready for the next run (every lane stores 0)
    }
    if (Qh == 1 || !c.out) return;
    // the last slice of sketch d to finish sums the slice terms
    int *cnt = a.cnt + c.cnt_sketch + d;
    __threadfence();
    __syncthreads();
    if (wg_atomic_ticket<P>(cnt, slot) != Qh - 1) return;
    __threadfence();
    sum_slices<Shape<P>::T>(c, d);
    atomicExch(cnt, 0);
}

template <int P>
__global__ __launch_bounds__(Shape<P>::T) void batch_kernel(BatchArgs a) {
    extern __shared__ float2 lds[];
    __shared__ int s_slot;
    for (;;) {
        const int t = wg_atomic_ticket<P>(a.head, &s_slot);
        if (t >= a.ntiles) break;
        batch_tile<P>(a, t, lds, &s_slot);
    }
    // every workgroup has taken its last queue ticket before it counts itself
    // here, so the last one may reset the queue for the next run
    if (threadIdx.x < 64) {
        const int v = atomicAdd(a.done, threadIdx.x == 0 ? 1 : 0);
        if (__builtin_amdgcn_readfirstlane(v) == (int)gridDim.x - 1) {
            atomicExch(a.head, 0);
            atomicExch(a.done, 0);
        }
    }
}

// Column maxima of every CP item's factors (the scales of the fixed-point
// count-sketch bins of its tiles) and the exponents of their norms (the
// scales of two modes packed into one transform), one wave per column.
// Entry k covers the R columns of one (item, mode); its columns are the
// global column indices [first, first + R), their maxima go to
// ws + out_off + r and their exponents to ws + out_off + exp_gap + r (floats).
struct AbsmaxEntry {
    const float *U;
    int64_t first;
    int64_t out_off;                 // in floats from the workspace base
    int64_t exp_gap;                 // N R of the item
    int I, R;
};

__global__ __launch_bounds__(256) void batch_absmax_kernel(const AbsmaxEntry *ent, int nent, int64_t ncols,
                                                           float *base) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= ncols) return;
    int lo = 0, hi = nent - 1;                   // last entry with first <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].first <= g) lo = mid;
        else hi = mid - 1;
    }
    const AbsmaxEntry e = ent[lo];
    const int64_t r = g - e.first;
    const float *u = e.U + r * e.I;
    constexpr int K = 8;
    float m = 0.f;
    double sq = 0.0;
    for (int i0 = lane; i0 < e.I; i0 += K * 64) {
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = i0 + k * 64 < e.I ? fabsf(u[i0 + k * 64]) : 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            m = (v[k] != v[k]) ? INFINITY : fmaxf(m, v[k]);
            sq += (double)v[k] * (double)v[k];
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        m = fmaxf(m, __shfl_xor(m, o));
        sq += __shfl_xor(sq, o);
    }
    if (lane == 0) {
        int ex = 0;
        if (m <= 3.4028234e38f && sq > 0.0) (void)frexp(sqrt(sq), &ex);
        base[e.out_off + r] = m;
        base[e.out_off + e.exp_gap + r] = (float)ex;
    }
}

template <typename K>
void allow_lds_batch(K kernel, size_t bytes) {
    fcs_allow_lds(reinterpret_cast<const void *>(kernel), bytes);
}

template <int P>
void launch_class(const BatchArgs &a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(batch_kernel<P>, dim3(grid), dim3(Shape<P>::T), lds, s, a);
}

template <int P>
void prepare_class(size_t lds) {
    allow_lds_batch(batch_kernel<P>, lds);
}

int threads_of(int P) { return P >= 1024 ? P / 16 : 64; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct fcs_batch {
    struct Cls {
        int P = 0;
        std::vector<BatchTile> tiles;
        size_t tiles_off = 0;
        size_t lds = 0;
        int grid = 0;
    };
    std::vector<CpDesc> desc;            // device pointers patched at prepare
    std::vector<int> cls_of;             // FFT size class of every item
    bool no_pack[NCLASS] = {};           // classes without two-mode packing
    std::vector<size_t> part_off, ytmp_off, kscr_off, umax_off;
    std::vector<AbsmaxEntry> absmax;     // column-max work, out_off patched at create
    size_t absmax_off = 0, umax_base = 0;
    int64_t absmax_cols = 0;
    std::vector<int> zero_items;         // CP items of rank 0
    Cls cls[NCLASS];
    size_t desc_off = 0, ctr_off = 0, total = 0;
    int nctr = 0;
    int64_t ntiles = 0;
    const void *prepared_ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *graph_ws = nullptr;
    hipStream_t cap[NCLASS + 1] = {};
    hipEvent_t ev[NCLASS + 1] = {};

    ~fcs_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &s : cap)
            if (s) (void)hipStreamDestroy(s);
    }
};

namespace {

int class_of(int64_t P) {
    int c = 0;
    while ((int64_t)FCS_MIN_FFT << c < P) ++c;
    return ((int64_t)FCS_MIN_FFT << c) == P && c < NCLASS ? c : -1;
}

// default persistent workgroups per CU of a class: as many as LDS holds, at most 8
int default_wpc(int P, size_t lds) {
    const int by_lds = (int)std::max<size_t>(1, (FCS_LDS_BYTES - 1024) / std::max<size_t>(lds + 64, 1));
    const int by_threads = std::max(1, 2048 / threads_of(P));
    return std::max(1, std::min({8, by_lds, by_threads}));
}

fcs_status launch_all(fcs_batch *b, char *ws, hipStream_t main, bool fork) {
    int *ctr = reinterpret_cast<int *>(ws + b->ctr_off);
    for (int it : b->zero_items) {
        const CpDesc &c = b->desc[it];
        if (c.out) {
            fcs_status st = fcs_zero_fill(c.out, (int64_t)c.D * c.Jt, main);
            if (st != FCS_OK) return st;
        }
        if (c.spec) {
            fcs_status st = fcs_zero_fill(reinterpret_cast<float *>(c.spec), (int64_t)c.D * c.s.Qh * c.s.P * 2, main);
            if (st != FCS_OK) return st;
        }
    }
    if (b->absmax_cols > 0) {
        const unsigned grid = (unsigned)fcs_ceil_div(b->absmax_cols, 4);
        hipLaunchKernelGGL(batch_absmax_kernel, dim3(grid), dim3(256), 0, main,
                           reinterpret_cast<const AbsmaxEntry *>(ws + b->absmax_off), (int)b->absmax.size(),
                           b->absmax_cols, reinterpret_cast<float *>(ws));
        FCS_LAUNCH_CHECK();
        // the class kernels (forked from ev[0] under capture) start after it
        if (fork) FCS_HIP_CHECK(hipEventRecord(b->ev[0], main));
    }
    int k = 0;
    for (int ci = 0; ci < NCLASS; ++ci) {
        fcs_batch::Cls &C = b->cls[ci];
        if (C.tiles.empty()) continue;
        BatchArgs a{};
        a.desc = reinterpret_cast<const CpDesc *>(ws + b->desc_off);
        a.tiles = reinterpret_cast<const BatchTile *>(ws + C.tiles_off);
        a.ntiles = (int)C.tiles.size();
        a.head = ctr + 2 * ci;
        a.done = ctr + 2 * ci + 1;
        a.cnt = ctr + 2 * NCLASS;
        hipStream_t s = main;
        if (fork) {
            s = b->cap[1 + k];
            FCS_HIP_CHECK(hipStreamWaitEvent(s, b->ev[0], 0));
        }
        FCS_DISPATCH_FFT(C.P, (launch_class<PP>(a, C.grid, C.lds, s)));
        FCS_LAUNCH_CHECK();
        if (fork) {
            FCS_HIP_CHECK(hipEventRecord(b->ev[1 + k], s));
            FCS_HIP_CHECK(hipStreamWaitEvent(main, b->ev[1 + k], 0));
        }
        ++k;
    }
    return FCS_OK;
}

}  // namespace

extern "C" fcs_status fcs_batch_create(const fcs_batch_item *items, int64_t count, const fcs_batch_config *cfg,
                                       fcs_batch_t *out) {
    fcs_clear_error();
    if (!out) FCS_FAIL(FCS_EINVAL, "null output pointer");
    if (count < 0 || (count > 0 && !items)) FCS_FAIL(FCS_EINVAL, "bad item array");
    if (count > INT32_MAX / FCS_MAX_D) FCS_FAIL(FCS_EUNSUPPORTED, "too many items");
    const int tile_ffts = (cfg && cfg->tile_ffts > 0) ? cfg->tile_ffts : 32;
    fcs_batch *b = new fcs_batch();
    for (int ci = 0; ci < NCLASS; ++ci) b->no_pack[ci] = cfg && cfg->no_pack[ci] != 0;
    std::vector<std::vector<double>> cost(NCLASS);
    for (int64_t i = 0; i < count; ++i) {
        const fcs_batch_item &it = items[i];
        const fcs_plan *p = it.plan;
        auto fail = [&](fcs_status st) {
            delete b;
            return st;
        };
        if (!p || !p->bound) return fail((fcs_set_error("item %lld: plan is null or not bound", (long long)i), FCS_EINVAL));
        if (p->P == 0) return fail((fcs_set_error("item %lld: no transform length fits", (long long)i), FCS_EUNSUPPORTED));
        const int ci = class_of(p->P);
        if (ci < 0) return fail((fcs_set_error("item %lld: FFT size %lld not built", (long long)i, (long long)p->P), FCS_EUNSUPPORTED));
        if (!it.out && !it.spec) return fail((fcs_set_error("item %lld: neither out nor spec", (long long)i), FCS_EINVAL));
        if (!it.U) return fail((fcs_set_error("item %lld: null factor array", (long long)i), FCS_EINVAL));
        CpDesc c{};
        desc_from_plan(c, p);
        c.out = it.out;
        c.spec = reinterpret_cast<float2 *>(it.spec);
        const double lg = std::log2((double)p->P);
        size_t part = 0, ytmp = 0, kscr = 0, umax = 0;
        if (it.kind == FCS_ITEM_KRON) {
            if (p->N != 4) return fail((fcs_set_error("item %lld: Kronecker item needs N=4", (long long)i), FCS_EINVAL));
            if (!it.U[0] || !it.U[1]) return fail((fcs_set_error("item %lld: null factor matrix", (long long)i), FCS_EINVAL));
            c.kind = FCS_DESC_KRON;
            if (cp_lds_bytes((int)p->P, c) > FCS_LDS_BYTES - 1024)
                return fail((fcs_set_error("item %lld: factor sketches exceed LDS", (long long)i), FCS_EUNSUPPORTED));
            c.U[0] = it.U[0];
            c.U[1] = it.U[1];
            c.R = 1;
            c.nchunks = c.rchunk = 1;
            kscr = (size_t)p->D * (p->J[0] + p->J[1] - 1 + p->J[2] + p->J[3] - 1) * sizeof(float);
            const double tc = 2.0 * ((double)p->I[0] * p->I[1] + (double)p->I[2] * p->I[3]) +
                              3.0 * p->Qh * p->P * lg;
            for (int d = 0; d < p->D; ++d) {
                b->cls[ci].tiles.push_back({(int32_t)i, d, 0, 0});
                cost[ci].push_back(tc);
            }
        } else if (it.kind == FCS_ITEM_CP) {
            if (it.R < 0) return fail((fcs_set_error("item %lld: R < 0", (long long)i), FCS_EINVAL));
            if (it.R > INT32_MAX) return fail((fcs_set_error("item %lld: R too large", (long long)i), FCS_EUNSUPPORTED));
            c.kind = FCS_DESC_CP;
            for (int n = 0; n < p->N; ++n)
                if (p->I[n] >= FCS_MAX_GATHER_INDEX)
                    return fail((fcs_set_error("item %lld: CP sketches need I_n < 2^30", (long long)i), FCS_EUNSUPPORTED));
            c.R = (int)it.R;
            c.lambda = it.lambda;
            if (it.R == 0) {
                c.nchunks = c.rchunk = 1;
                b->zero_items.push_back((int)i);
            } else {
                for (int n = 0; n < p->N; ++n) {
                    if (!it.U[n]) return fail((fcs_set_error("item %lld: null factor %d", (long long)i, n), FCS_EINVAL));
                    c.U[n] = it.U[n];
                    // out_off is the item-relative offset until the layout is known
                    b->absmax.push_back({it.U[n], b->absmax_cols, (int64_t)n * it.R, (int64_t)p->N * it.R,
                                         (int)p->I[n], (int)it.R});
                    b->absmax_cols += it.R;
                }
                umax = 2 * (size_t)p->N * it.R * sizeof(float);
                c.rchunk = (int)std::min<int64_t>(it.R, std::max<int64_t>(1, fcs_ceil_div(tile_ffts, p->N)));
                c.nchunks = (int)fcs_ceil_div(it.R, c.rchunk);
                // per rank and mode: the count sketch (entries and bins)
                // and one transform, except on the conjugate-symmetric
                // slices, where two modes share a transform
                double scat = 0.0;
                int folded = 0;
                for (int n = 0; n < p->N; ++n) {
                    scat += 4.0 * std::max<int64_t>(p->I[n], p->P);
                    folded += p->J[n] > p->P;
                }
                auto per_rank = [&](int q) {
                    const bool packs = folded == 0 && (q == 0 || 2 * q == p->Q);
                    const int ffts = packs ? (p->N + 1) / 2 : p->N;
                    return scat + ffts * p->P * lg;
                };
                if (c.nchunks > 1) {
                    c.cnt_slice = b->nctr;
                    b->nctr += p->D * p->Qh;
                    part = (size_t)p->D * p->Qh * c.nchunks * p->P * sizeof(float2);
                }
                if (p->Qh > 1 && it.out) {
                    c.cnt_sketch = b->nctr;
                    b->nctr += p->D;
                    ytmp = (size_t)p->D * p->Qh * p->Jt * sizeof(float);
                }
                for (int d = 0; d < p->D; ++d)
                    for (int q = 0; q < p->Qh; ++q)
                        for (int ch = 0; ch < c.nchunks; ++ch) {
                            const int nr = std::min(c.R, (ch + 1) * c.rchunk) - ch * c.rchunk;
                            b->cls[ci].tiles.push_back({(int32_t)i, d, q, ch});
                            cost[ci].push_back(nr * per_rank(q));
                        }
            }
        } else {
            return fail((fcs_set_error("item %lld: unknown kind %d", (long long)i, it.kind), FCS_EINVAL));
        }
        b->cls[ci].P = (int)p->P;
        b->cls[ci].lds = std::max(b->cls[ci].lds, cp_lds_bytes((int)p->P, c));
        b->desc.push_back(c);
        b->cls_of.push_back(ci);
        b->part_off.push_back(part);
        b->ytmp_off.push_back(ytmp);
        b->kscr_off.push_back(kscr);
        b->umax_off.push_back(umax);
    }
    // costliest tiles first in every class
    const int cus = fcs_device_cu_count();
    for (int ci = 0; ci < NCLASS; ++ci) {
        fcs_batch::Cls &C = b->cls[ci];
        if (C.tiles.empty()) continue;
        std::vector<size_t> order(C.tiles.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[ci][x] > cost[ci][y]; });
        std::vector<BatchTile> sorted(order.size());
        for (size_t k = 0; k < order.size(); ++k) sorted[k] = C.tiles[order[k]];
        C.tiles.swap(sorted);
        int wpc = (cfg && cfg->wg_per_cu[ci] > 0) ? cfg->wg_per_cu[ci] : default_wpc(C.P, C.lds);
        C.grid = (int)std::min<int64_t>((int64_t)C.tiles.size(), (int64_t)wpc * cus);
        b->ntiles += (int64_t)C.tiles.size();
    }
    // workspace: descriptors, tile lists, counters, partial spectra, Kronecker scratch
    size_t cur = 0;
    b->desc_off = cur;
    cur = align256(cur + b->desc.size() * sizeof(CpDesc));
    for (int ci = 0; ci < NCLASS; ++ci) {
        b->cls[ci].tiles_off = cur;
        cur = align256(cur + b->cls[ci].tiles.size() * sizeof(BatchTile));
    }
    b->ctr_off = cur;
    cur = align256(cur + (size_t)(2 * NCLASS + b->nctr) * sizeof(int));
    for (size_t i = 0; i < b->desc.size(); ++i) {
        const size_t po = b->part_off[i], yo = b->ytmp_off[i], ko = b->kscr_off[i];
        b->part_off[i] = po ? cur : 0;
        cur = align256(cur + po);
        b->ytmp_off[i] = yo ? cur : 0;
        cur = align256(cur + yo);
        b->kscr_off[i] = ko ? cur : 0;
        cur = align256(cur + ko);
    }
    // column maxima of the CP items (4-byte aligned, packed) and the
    // column-max work list
    b->umax_base = cur;
    for (size_t i = 0, e = 0; i < b->desc.size(); ++i) {
        const size_t uo = b->umax_off[i];
        b->umax_off[i] = uo ? cur : 0;
        if (uo) {
            for (int n = 0; n < b->desc[i].N; ++n, ++e) b->absmax[e].out_off += (int64_t)(cur / sizeof(float));
        }
        cur += uo;
    }
    cur = align256(cur);
    b->absmax_off = cur;
    cur = align256(cur + b->absmax.size() * sizeof(AbsmaxEntry));
    b->total = std::max<size_t>(cur, 256);
    *out = b;
    return FCS_OK;
}

extern "C" size_t fcs_batch_workspace_bytes(fcs_batch_t b) { return b ? b->total : 0; }

extern "C" fcs_status fcs_batch_info(fcs_batch_t b, int64_t *tiles, int32_t *grids) {
    fcs_clear_error();
    if (!b) FCS_FAIL(FCS_EINVAL, "null batch");
    if (tiles) *tiles = b->ntiles;
    if (grids)
        for (int ci = 0; ci < NCLASS; ++ci) grids[ci] = b->cls[ci].tiles.empty() ? 0 : b->cls[ci].grid;
    return FCS_OK;
}

extern "C" fcs_status fcs_batch_prepare(fcs_batch_t b, void *ws, size_t ws_bytes, void *stream) {
    fcs_clear_error();
    if (!b) FCS_FAIL(FCS_EINVAL, "null batch");
    if (!ws || ws_bytes < b->total) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, b->total);
    if (!fcs_aligned(ws, 256)) FCS_FAIL(FCS_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *w = static_cast<char *>(ws);
    for (size_t i = 0; i < b->desc.size(); ++i) {
        b->desc[i].partial = b->part_off[i] ? reinterpret_cast<float2 *>(w + b->part_off[i]) : nullptr;
        b->desc[i].ytmp = b->ytmp_off[i] ? reinterpret_cast<float *>(w + b->ytmp_off[i]) : nullptr;
        b->desc[i].kscratch = b->kscr_off[i] ? reinterpret_cast<float *>(w + b->kscr_off[i]) : nullptr;
        b->desc[i].umax = b->umax_off[i] ? reinterpret_cast<const float *>(w + b->umax_off[i]) : nullptr;
        // without the norm exponents the tiles transform every mode alone
        b->desc[i].uexp = (b->desc[i].umax && !b->no_pack[b->cls_of[i]])
                              ? b->desc[i].umax + (int64_t)b->desc[i].N * b->desc[i].R
                              : nullptr;
    }
    if (!b->absmax.empty())
        FCS_HIP_CHECK(hipMemcpyAsync(w + b->absmax_off, b->absmax.data(), b->absmax.size() * sizeof(AbsmaxEntry),
                                     hipMemcpyHostToDevice, s));
    if (!b->desc.empty())
        FCS_HIP_CHECK(hipMemcpyAsync(w + b->desc_off, b->desc.data(), b->desc.size() * sizeof(CpDesc),
                                     hipMemcpyHostToDevice, s));
    for (int ci = 0; ci < NCLASS; ++ci) {
        const auto &C = b->cls[ci];
        if (!C.tiles.empty())
            FCS_HIP_CHECK(hipMemcpyAsync(w + C.tiles_off, C.tiles.data(), C.tiles.size() * sizeof(BatchTile),
                                         hipMemcpyHostToDevice, s));
    }
    const int64_t nctr = 2 * NCLASS + b->nctr;
    fcs_status st = fcs_zero_fill(reinterpret_cast<float *>(w + b->ctr_off), nctr, s);
    if (st != FCS_OK) return st;
    // the host copies must stay valid until the transfers are done
    FCS_HIP_CHECK(hipStreamSynchronize(s));
    for (int ci = 0; ci < NCLASS; ++ci)
        if (!b->cls[ci].tiles.empty()) FCS_DISPATCH_FFT(b->cls[ci].P, (prepare_class<PP>(b->cls[ci].lds)));
    b->prepared_ws = ws;
    return FCS_OK;
}

extern "C" fcs_status fcs_batch_run(fcs_batch_t b, void *ws, size_t ws_bytes, int32_t use_graph, void *stream) {
    fcs_clear_error();
    if (!b) FCS_FAIL(FCS_EINVAL, "null batch");
    if (!ws || ws_bytes < b->total) FCS_FAIL(FCS_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, b->total);
    if (ws != b->prepared_ws) FCS_FAIL(FCS_EINVAL, "workspace was not prepared with fcs_batch_prepare");
    hipStream_t s = (hipStream_t)stream;
    char *w = static_cast<char *>(ws);
    if (b->ntiles == 0 && b->zero_items.empty()) return FCS_OK;
    if (!use_graph) return launch_all(b, w, s, false);
    if (!b->exec || b->graph_ws != ws) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        for (int k = 0; k <= NCLASS; ++k) {
            if (!b->cap[k]) FCS_HIP_CHECK(hipStreamCreateWithFlags(&b->cap[k], hipStreamNonBlocking));
            if (!b->ev[k]) FCS_HIP_CHECK(hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming));
        }
        // capture on private streams: the class kernels are forked from one
        // origin and joined back, so the graph runs them concurrently
        FCS_HIP_CHECK(hipStreamBeginCapture(b->cap[0], hipStreamCaptureModeThreadLocal));
        fcs_status st = FCS_OK;
        if (hipEventRecord(b->ev[0], b->cap[0]) != hipSuccess) {
            fcs_set_error("event record during capture failed");
            st = FCS_EDEVICE;
        }
        if (st == FCS_OK) st = launch_all(b, w, b->cap[0], true);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap[0], &g);
        if (st != FCS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) FCS_FAIL(FCS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        b->graph = g;
        FCS_HIP_CHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_ws = ws;
    }
    FCS_HIP_CHECK(hipGraphLaunch(b->exec, s));
    return FCS_OK;
}

extern "C" fcs_status fcs_batch_destroy(fcs_batch_t b) {
    fcs_clear_error();
    delete b;
    return FCS_OK;
}
