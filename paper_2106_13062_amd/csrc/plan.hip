// Plans: validation, sizes, seeded hash tables and twiddle tables on the
// device, status strings and small shared launch helpers.
#include "fcs_internal.h"

#include <map>
#include <mutex>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>
#include <vector>

// ---------------------------------------------------------------------------
// error state (per host thread)
// ---------------------------------------------------------------------------
static thread_local char g_err[512];

void fcs_set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void fcs_clear_error() { g_err[0] = '\0'; }

extern "C" const char *fcs_last_error(void) { return g_err; }

extern "C" const char *fcs_status_str(fcs_status s) {
    switch (s) {
    case FCS_OK: return "FCS_OK";
    case FCS_EINVAL: return "FCS_EINVAL: invalid argument";
    case FCS_ENOMEM: return "FCS_ENOMEM: caller buffer too small";
    case FCS_EADMIT: return "FCS_EADMIT: rejected by the admission bound";
    case FCS_EDEVICE: return "FCS_EDEVICE: HIP call or kernel launch failed";
    case FCS_EUNSUPPORTED: return "FCS_EUNSUPPORTED: outside this build's limits";
    }
    return "unknown fcs_status";
}

void fcs_allow_lds(const void *kernel, size_t bytes) {
    if (bytes <= 65536) return;
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    size_t &have = done[{kernel, dev}];
    if (have >= bytes) return;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        have = bytes;
}

int fcs_device_cu_count() {
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cu = prop.multiProcessorCount;
    }
    return cu;
}

// ---------------------------------------------------------------------------
// device hash family: SplitMix64 output function (Steele, Lea, Flood 2014)
// ---------------------------------------------------------------------------
__host__ __device__ static inline uint64_t sm64_mix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct HashArgs {
    uint32_t *tab;
    uint64_t seed_mixed;   // mix(seed)
    int64_t off[FCS_MAX_ORDER + 1];
    int64_t J[FCS_MAX_ORDER];      // hash range Jh_n of the multiply-shift
    int64_t hmul[FCS_MAX_ORDER];   // multiplier of the hash values
    int N;
    int64_t sumI;
    int64_t total;         // D * sumI
};

__global__ void hash_tables_kernel(HashArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.total) return;
    const int64_t d = t / a.sumI;
    const int64_t e = t - d * a.sumI;
    int n = 0;
    while (n + 1 < a.N && e >= a.off[n + 1]) ++n;
    const int64_t i = e - a.off[n];
    const uint64_t key = sm64_mix(a.seed_mixed + ((uint64_t)d << 16) + (uint64_t)n);
    const uint64_t y = sm64_mix(key + (uint64_t)i);
    const uint64_t h = (((y >> 32) * (uint64_t)a.J[n]) >> 32) * (uint64_t)a.hmul[n];
    a.tab[t] = (uint32_t)h | ((y & 1ull) ? FCS_S_BIT : 0u);
}

// exp(-2 pi i k / n) in single precision.  The angle 2 pi k / n is reduced
// exactly, in integers, to an octant o and a remainder r (8k = o n + r,
// 0 <= r < n); sincospif gives the sine and cosine of pi r / (4n) (pi (n - r)
// / (4n), the complement, in odd octants), and the quarter-turn symmetries
// place them.  n <= 2^20, so 4n and r are exact in float and the argument
// is rounded once.
__global__ void twiddle_kernel(float2 *w, int64_t n64) {
    const int64_t k64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k64 >= n64) return;
    const int n = (int)n64;
    const int k = (int)k64;
    const int o = (8 * k) / n;
    const int r = 8 * k - o * n;
    float sb, cb;      // sine and cosine of the angle past the quarter turn
    if (o & 1) {
        sincospif((float)(n - r) / (float)(4 * n), &cb, &sb);
    } else {
        sincospif((float)r / (float)(4 * n), &sb, &cb);
    }
    float c, s;
    switch (o >> 1) {
    case 0: c = cb; s = sb; break;
    case 1: c = -sb; s = cb; break;
    case 2: c = -cb; s = -sb; break;
    default: c = sb; s = -cb; break;
    }
    w[k] = make_float2(c, -s);
}

__global__ void zero_fill_kernel(float4 *p4, int64_t n4, float *tail, int64_t ntail) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n4; k += stride)
        p4[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < ntail) tail[k] = 0.f;
}

fcs_status fcs_zero_fill(float *p, int64_t n, hipStream_t s) {
    if (n <= 0) return FCS_OK;
    // align the vector part to 16 bytes
    int64_t head = 0;
    while (head < n && !fcs_aligned(p + head, 16)) ++head;
    if (head > 0) {
        zero_fill_kernel<<<1, 64, 0, s>>>(nullptr, 0, p, head);
        FCS_LAUNCH_CHECK();
    }
    const int64_t n4 = (n - head) / 4;
    const int64_t ntail = (n - head) - n4 * 4;
    int64_t blocks = std::min<int64_t>(fcs_ceil_div(std::max<int64_t>(n4, 1), 256), 4096);
    zero_fill_kernel<<<(unsigned)blocks, 256, 0, s>>>(reinterpret_cast<float4 *>(p + head), n4,
                                                     p + head + n4 * 4, ntail);
    FCS_LAUNCH_CHECK();
    return FCS_OK;
}

// ---------------------------------------------------------------------------
// transform length: L = Q * P, P a power of two in [FCS_MIN_FFT, FCS_MAX_FFT]
// ---------------------------------------------------------------------------
static double cp_cost(const fcs_plan *p, int64_t P, int Q) {
    // per (sketch, rank) and stored slice: for each mode a count sketch over
    // its I_n entries and J_n buckets (weight 16 per entry or bucket against
    // one FFT point and radix-2 stage: the measured optimum of the batch
    // autotuner's length model) and one P-point FFT, except on the
    // conjugate-symmetric slices (q = 0 and, Q even, Q/2), where two modes
    // share a transform when no hash is folded; plus the inverse of the slice
    const int Qh = Q / 2 + 1;
    const double lg = std::log2((double)P);
    const double fft = (double)P * lg;
    double sketch = 0.0;
    bool folded = false;
    for (int n = 0; n < p->N; ++n) {
        sketch += 16.0 * (double)(p->J[n] + p->I[n]);
        folded = folded || p->J[n] > P;
    }
    const int nself = (Q % 2 == 0 && Q > 1) ? 2 : 1;
    const int packed = folded ? p->N : (p->N + 1) / 2;
    return (double)Qh * (sketch + fft) + fft * ((double)nself * packed + (double)(Qh - nself) * p->N);
}

static bool choose_transform(fcs_plan *p, int64_t Lreq) {
    if (Lreq > 0) {
        for (int64_t P = FCS_MAX_FFT; P >= FCS_MIN_FFT; P /= 2) {
            if (Lreq % P) continue;
            int64_t Q = Lreq / P;
            if (Q >= 1 && Q <= 64) {
                p->P = P;
                p->Q = (int)Q;
                p->L = Lreq;
                return true;
            }
        }
        return false;
    }
    double best = 0.0;
    bool found = false;
    for (int64_t P = FCS_MIN_FFT; P <= FCS_MAX_FFT; P *= 2) {
        int64_t Q = fcs_ceil_div(p->Jt, P);
        if (Q > 64) continue;
        double c = cp_cost(p, P, (int)Q);
        if (!found || c < best) {
            best = c;
            found = true;
            p->P = P;
            p->Q = (int)Q;
            p->L = P * Q;
        }
    }
    return found;
}

static fcs_status plan_create(const fcs_plan_desc *desc, fcs_plan_t *out, bool hcs) {
    if (!desc || !out) FCS_FAIL(FCS_EINVAL, "null description or output pointer");
    if (desc->N < 1 || desc->N > FCS_MAX_ORDER)
        FCS_FAIL(FCS_EINVAL, "order N=%d outside [1, %d]", desc->N, FCS_MAX_ORDER);
    if (!desc->I || !desc->J) FCS_FAIL(FCS_EINVAL, "null I or J array");
    if (desc->D < 1 || desc->D > FCS_MAX_D)
        FCS_FAIL(FCS_EINVAL, "D=%d outside [1, %d]", desc->D, FCS_MAX_D);
    fcs_plan tmp;
    tmp.N = desc->N;
    tmp.D = desc->D;
    tmp.seed = desc->seed;
    double prodI = 1.0;
    int64_t sumJ = 0;
    for (int n = 0; n < tmp.N; ++n) {
        if (desc->I[n] < 1) FCS_FAIL(FCS_EINVAL, "I[%d]=%lld < 1", n, (long long)desc->I[n]);
        if (desc->J[n] < 1) FCS_FAIL(FCS_EINVAL, "J[%d]=%lld < 1", n, (long long)desc->J[n]);
        if (desc->I[n] > INT32_MAX) FCS_FAIL(FCS_EUNSUPPORTED, "I[%d] exceeds 2^31-1", n);
        if (desc->J[n] > INT32_MAX) FCS_FAIL(FCS_EUNSUPPORTED, "J[%d] exceeds 2^31-1", n);
        tmp.I[n] = desc->I[n];
        tmp.Jh[n] = desc->J[n];
        tmp.off[n] = tmp.sumI;
        tmp.sumI += desc->I[n];
        prodI *= (double)desc->I[n];
    }
    if (prodI >= 4.6e18) FCS_FAIL(FCS_EUNSUPPORTED, "tensor has 2^62 or more entries");
    tmp.hcs = hcs;
    int64_t mul = 1;
    for (int n = 0; n < tmp.N; ++n) {
        tmp.hmul[n] = hcs ? mul : 1;
        tmp.J[n] = (tmp.Jh[n] - 1) * tmp.hmul[n] + 1;
        sumJ += tmp.J[n];
        if (hcs) {
            mul *= tmp.Jh[n];
            if (mul >= ((int64_t)1 << 31) - 1)
                FCS_FAIL(FCS_EUNSUPPORTED, "prod J_n exceeds 2^31 - 2 for a higher-order count sketch");
        }
    }
    tmp.Jt = sumJ - tmp.N + 1;
    if (tmp.Jt >= ((int64_t)1 << 31) - 1) FCS_FAIL(FCS_EUNSUPPORTED, "J~ = %lld too large", (long long)tmp.Jt);
    if (desc->L != 0) {
        if (desc->L < tmp.Jt)
            FCS_FAIL(FCS_EINVAL, "L=%lld is smaller than J~=%lld", (long long)desc->L, (long long)tmp.Jt);
        if (!choose_transform(&tmp, desc->L))
            FCS_FAIL(FCS_EUNSUPPORTED, "L=%lld is not Q*P with P a power of two in [%d,%d] and Q<=64",
                     (long long)desc->L, FCS_MIN_FFT, FCS_MAX_FFT);
    } else if (!choose_transform(&tmp, 0)) {
        // very long sketches: the dense, COO and inner-product paths still work
        tmp.P = 0;
        tmp.Q = 0;
        tmp.L = 0;
    }
    tmp.Qh = tmp.Q / 2 + 1;
    // device layout: packed hash words, then twiddles, each 256-byte aligned
    auto align256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    tmp.tab_off = 0;
    size_t cur = align256((size_t)tmp.D * (size_t)tmp.sumI * sizeof(uint32_t));
    tmp.twP_off = cur;
    cur = align256(cur + (size_t)tmp.P * sizeof(float2));
    tmp.twL_off = cur;
    cur = align256(cur + (size_t)tmp.L * sizeof(float2));
    tmp.iblock = 0;
    for (int n = 0; n < tmp.N; ++n) {
        tmp.ioff[n] = tmp.iblock;
        tmp.iblock += tmp.J[n] + 1 + tmp.I[n] + 2 * tmp.J[n];
    }
    tmp.inv_off = cur;
    cur = align256(cur + (size_t)tmp.D * (size_t)tmp.iblock * sizeof(int32_t));
    tmp.perm_off = cur;
    tmp.perm_bytes = fcs_dense_perm_bytes(&tmp);
    cur = align256(cur + tmp.perm_bytes);
    tmp.total = cur;
    fcs_plan *p = new (std::nothrow) fcs_plan(tmp);
    if (!p) FCS_FAIL(FCS_ENOMEM, "host allocation of the plan failed");
    *out = p;
    return FCS_OK;
}

extern "C" fcs_status fcs_plan_create(const fcs_plan_desc *desc, fcs_plan_t *out) {
    fcs_clear_error();
    return plan_create(desc, out, false);
}

extern "C" fcs_status fcs_plan_create_hcs(const fcs_plan_desc *desc, fcs_plan_t *out) {
    fcs_clear_error();
    return plan_create(desc, out, true);
}

extern "C" size_t fcs_plan_table_bytes(fcs_plan_t p) { return p ? p->total : 0; }

// Inverse hash lists (bucket offsets and entries per sketch and mode),
// computed with the same hash function on the host and copied to the
// plan's table memory.  Synchronises the stream.
static fcs_status build_inverse(const fcs_plan *p, int32_t *dev_inv, hipStream_t s) {
    std::vector<int32_t> host((size_t)p->D * (size_t)p->iblock);
    const uint64_t sm = sm64_mix(p->seed);
    for (int d = 0; d < p->D; ++d) {
        for (int n = 0; n < p->N; ++n) {
            int32_t *blk = host.data() + (size_t)d * p->iblock + p->ioff[n];
            const int64_t In = p->I[n], Jn = p->J[n], Jh = p->Jh[n], hm = p->hmul[n];
            int32_t *off = blk;
            int32_t *ent = blk + Jn + 1;
            std::vector<uint32_t> word((size_t)In);
            const uint64_t key = sm64_mix(sm + ((uint64_t)d << 16) + (uint64_t)n);
            for (int64_t j = 0; j <= Jn; ++j) off[j] = 0;
            for (int64_t i = 0; i < In; ++i) {
                const uint64_t y = sm64_mix(key + (uint64_t)i);
                const uint32_t h = (uint32_t)((((y >> 32) * (uint64_t)Jh) >> 32) * (uint64_t)hm);
                word[(size_t)i] = h | ((y & 1ull) ? FCS_S_BIT : 0u);
                off[h + 1] += 1;
            }
            for (int64_t j = 0; j < Jn; ++j) off[j + 1] += off[j];
            std::vector<int32_t> fill(off, off + Jn);
            for (int64_t i = 0; i < In; ++i) {
                const uint32_t w = word[(size_t)i];
                const uint32_t h = w & FCS_H_MASK;
                ent[fill[h]++] = (int32_t)((uint32_t)i | (w & FCS_S_BIT));
            }
            // first- and second-entry words (indices >= 2^30 are not
            // gathered this way: the CP paths reject such modes)
            int32_t *first = ent + In;
            int32_t *second = first + Jn;
            for (int64_t j = 0; j < Jn; ++j) {
                const int32_t c = off[j + 1] - off[j];
                uint32_t f = FCS_FIRST_EMPTY, g = FCS_FIRST_EMPTY;
                if (c > 0) {
                    const uint32_t e = (uint32_t)ent[off[j]];
                    f = (e & FCS_IDX_MASK) | (e & FCS_S_BIT) | (c > 1 ? FCS_MORE_BIT : 0u);
                }
                if (c > 1) {
                    const uint32_t e = (uint32_t)ent[off[j] + 1];
                    g = (e & FCS_IDX_MASK) | (e & FCS_S_BIT) | (c > 2 ? FCS_MORE_BIT : 0u);
                }
                first[j] = (int32_t)f;
                second[j] = (int32_t)g;
            }
        }
    }
    FCS_HIP_CHECK(hipMemcpyAsync(dev_inv, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    FCS_HIP_CHECK(hipStreamSynchronize(s));
    return FCS_OK;
}

void fcs_mode0_hashes(const fcs_plan *p, uint32_t *h0) {
    const uint64_t sm = sm64_mix(p->seed);
    for (int d = 0; d < p->D; ++d) {
        const uint64_t key = sm64_mix(sm + ((uint64_t)d << 16) + 0u);
        for (int64_t i = 0; i < p->I[0]; ++i) {
            const uint64_t y = sm64_mix(key + (uint64_t)i);
            h0[(size_t)d * p->I[0] + i] = (uint32_t)((((y >> 32) * (uint64_t)p->Jh[0]) >> 32) * (uint64_t)p->hmul[0]);
        }
    }
}

// Largest multiplicity of h_0 values over all sketches, evaluated with the
// same hash function on the host (small plans only).
static int mode0_multiplicity(const fcs_plan *p) {
    const int64_t I0 = p->I[0];
    if ((double)I0 * (double)p->D > 268435456.0) return INT32_MAX;
    const uint64_t sm = sm64_mix(p->seed);
    std::vector<uint32_t> h((size_t)I0);
    int best = 0;
    for (int d = 0; d < p->D; ++d) {
        const uint64_t key = sm64_mix(sm + ((uint64_t)d << 16) + 0u);
        for (int64_t i = 0; i < I0; ++i) {
            const uint64_t y = sm64_mix(key + (uint64_t)i);
            h[(size_t)i] = (uint32_t)((((y >> 32) * (uint64_t)p->Jh[0]) >> 32) * (uint64_t)p->hmul[0]);
        }
        std::sort(h.begin(), h.end());
        int run = 1;
        for (size_t i = 1; i <= h.size(); ++i) {
            if (i < h.size() && h[i] == h[i - 1]) {
                ++run;
            } else {
                best = std::max(best, run);
                run = 1;
            }
        }
    }
    return std::max(best, 1);
}

extern "C" fcs_status fcs_plan_bind(fcs_plan_t p, void *dev_tables, void *stream) {
    fcs_clear_error();
    if (!p) FCS_FAIL(FCS_EINVAL, "null plan");
    if (!dev_tables) FCS_FAIL(FCS_EINVAL, "null table buffer");
    if (!fcs_aligned(dev_tables, 256)) FCS_FAIL(FCS_EINVAL, "table buffer not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)dev_tables;
    HashArgs a;
    a.tab = (uint32_t *)(base + p->tab_off);
    a.seed_mixed = sm64_mix(p->seed);
    for (int n = 0; n < FCS_MAX_ORDER + 1; ++n) a.off[n] = (n < p->N) ? p->off[n] : p->sumI;
    for (int n = 0; n < FCS_MAX_ORDER; ++n) {
        a.J[n] = (n < p->N) ? p->Jh[n] : 1;
        a.hmul[n] = (n < p->N) ? p->hmul[n] : 1;
    }
    a.N = p->N;
    a.sumI = p->sumI;
    a.total = (int64_t)p->D * p->sumI;
    hash_tables_kernel<<<(unsigned)fcs_ceil_div(a.total, 256), 256, 0, s>>>(a);
    FCS_LAUNCH_CHECK();
    if (p->P > 0) {
        twiddle_kernel<<<(unsigned)fcs_ceil_div(p->P, 256), 256, 0, s>>>((float2 *)(base + p->twP_off), p->P);
        FCS_LAUNCH_CHECK();
        twiddle_kernel<<<(unsigned)fcs_ceil_div(p->L, 256), 256, 0, s>>>((float2 *)(base + p->twL_off), p->L);
        FCS_LAUNCH_CHECK();
    }
    p->m0 = mode0_multiplicity(p);
    {
        fcs_status st = build_inverse(p, (int32_t *)(base + p->inv_off), s);
        if (st != FCS_OK) return st;
    }
    p->perm = p->perm_bytes ? (const uint8_t *)(base + p->perm_off) : nullptr;
    p->perm_ready = false;
    p->inv = (const int32_t *)(base + p->inv_off);
    p->tab = (const uint32_t *)(base + p->tab_off);
    p->twP = (const float2 *)(base + p->twP_off);
    p->twL = (const float2 *)(base + p->twL_off);
    p->bound = true;
    return FCS_OK;
}

extern "C" size_t fcs_plan_dense_order_bytes(fcs_plan_t p) { return p ? p->perm_bytes : 0; }

extern "C" fcs_status fcs_plan_dense_order(fcs_plan_t p, uint8_t *out, size_t bytes, int32_t *group_size) {
    fcs_clear_error();
    if (!p) FCS_FAIL(FCS_EINVAL, "null plan");
    if (p->perm_bytes && !out) FCS_FAIL(FCS_EINVAL, "null output");
    if (bytes < p->perm_bytes) FCS_FAIL(FCS_EINVAL, "output of %zu bytes, %zu needed", bytes, p->perm_bytes);
    fcs_plan tmp = *p;           // the bind-time bound m0 on a copy
    tmp.m0 = mode0_multiplicity(&tmp);
    if (group_size) *group_size = fcs_dense_group_size(&tmp);
    if (!p->perm_bytes) return FCS_OK;
    std::vector<uint32_t> h0((size_t)p->D * (size_t)p->I[0]);
    fcs_mode0_hashes(&tmp, h0.data());
    fcs_dense_lane_order(&tmp, h0.data(), out);
    return FCS_OK;
}

extern "C" fcs_status fcs_plan_export(fcs_plan_t p, int32_t d, int32_t n, int32_t *h_host,
                                      int8_t *s_host, void *stream) {
    fcs_clear_error();
    if (!p || !p->bound) FCS_FAIL(FCS_EINVAL, "plan is null or not bound");
    if (d < 0 || d >= p->D || n < 0 || n >= p->N) FCS_FAIL(FCS_EINVAL, "d or n out of range");
    if (!h_host || !s_host) FCS_FAIL(FCS_EINVAL, "null host output");
    const int64_t cnt = p->I[n];
    uint32_t *tmp = new (std::nothrow) uint32_t[cnt];
    if (!tmp) FCS_FAIL(FCS_ENOMEM, "host allocation failed");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(tmp, p->tab + (int64_t)d * p->sumI + p->off[n], cnt * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete[] tmp;
        FCS_FAIL(FCS_EDEVICE, "table copy failed: %s", hipGetErrorString(e));
    }
    for (int64_t i = 0; i < cnt; ++i) {
        h_host[i] = (int32_t)(tmp[i] & FCS_H_MASK);
        s_host[i] = (tmp[i] & FCS_S_BIT) ? -1 : 1;
    }
    delete[] tmp;
    return FCS_OK;
}

extern "C" fcs_status fcs_plan_info(fcs_plan_t p, int64_t *Jtilde, int64_t *L, int64_t *P, int32_t *Q) {
    fcs_clear_error();
    if (!p) FCS_FAIL(FCS_EINVAL, "null plan");
    if (Jtilde) *Jtilde = p->Jt;
    if (L) *L = p->L;
    if (P) *P = p->P;
    if (Q) *Q = p->Q;
    return FCS_OK;
}

extern "C" int64_t fcs_plan_spec_len(fcs_plan_t p) {
    if (!p || p->P == 0) return 0;
    return (int64_t)p->Qh * p->P;
}

extern "C" fcs_status fcs_plan_destroy(fcs_plan_t p) {
    delete p;
    return FCS_OK;
}

extern "C" size_t fcs_workspace_bytes(fcs_plan_t p, int32_t op, int64_t R, int64_t P) {
    if (!p) return 0;
    switch (op) {
    case FCS_OP_DENSE: return fcs_ws_dense(p);
    case FCS_OP_COO: return fcs_ws_coo(p);
    case FCS_OP_CP: return fcs_ws_cp(p, R);
    case FCS_OP_INNER: return fcs_ws_inner(p);
    case FCS_OP_FREE_MODE: return fcs_ws_free_mode(p, P);
    case FCS_OP_SPECTRUM: return fcs_ws_spectrum(p);
    case FCS_OP_KRON: return fcs_ws_kron(p);
    case FCS_OP_CONTRACTION: return fcs_ws_contraction(p, R);
    case FCS_OP_FULL: return fcs_ws_full(p, P);
    default: return 0;
    }
}
