// cube_select.hip -- exact selection (k-th smallest valid voxel) and the
// median by histogram refinement: the global, multi-pass median task the
// paper names in Section 3.
//
// Every valid voxel maps to a 32-bit key that orders like the value (-0
// before +0): key = bits ^ (sign ? 0xffffffff : 0x80000000).  Three passes
// histogram the key 12, 12 and 8 bits at a time; in each pass only voxels
// whose key starts with the prefix chosen so far are counted.  The last
// block of a pass scans that pass's histogram, picks the bin holding the
// wanted rank, extends the prefix and lowers the rank, on the device, so the
// host never waits between passes.  After the third pass the prefix is the
// whole key of the selected voxel.  For the median of an even count the
// upper middle comes from the same passes (the same key again, or the next
// non-empty key of the last histogram) or, failing both, from one more pass
// that takes the smallest valid key above the lower middle.  Counting uses the same lane-interleaved
// LDS sub-histograms as the statistics pass, flushed with one 64-bit atomic
// per non-empty bin per block.
#include <string.h>

#include <mutex>

#include "cube_scan.h"

namespace cube {

struct SelectState {
    unsigned long long rank;     // rank still wanted inside the prefix bucket
    unsigned long long n_valid;  // valid voxels (set by the first pass)
    unsigned int prefix;         // key bits chosen so far
    unsigned int error;          // 1: rank >= n_valid
    float value;                 // the selected voxel (after the last pass)
    unsigned int rank_mode;      // 0: `rank` as given; 1: the median, rank
                                 // (n_valid - 1) / 2 set once n_valid is known
    unsigned int want_next;      // also find the voxel of the next rank
    unsigned int need_next;      // ...which the last histogram did not hold
    unsigned int next_key;       // smallest key above the selected one (min)
    float value_next;            // the voxel of the next rank
    unsigned int collect;        // pass 1 copies the first pass's bucket out
    unsigned int overflow;       // ...and a block's region overflowed
};

struct SelectArgs {
    Geom g;
    int32_t pass, copies_log2;
    SelectState *st;
    unsigned long long *acc;     // 4096 accumulators, zero between passes
    unsigned int *ticket;
    float *out;                  // optional device copy of the result
    float *cand;                 // per-block candidate regions, cand_cap floats each
    unsigned int *cand_n;        // voxels each block copied (pass 1)
    unsigned int cand_cap;
    Claim claim;                 // the partition of the full-box passes
};

// Pass p histograms key bits [shift, shift + width): widths 12, 12, 8.
__host__ __device__ __forceinline__ int sel_width(int p) { return p == 2 ? 8 : 12; }
__host__ __device__ __forceinline__ int sel_shift(int p) { return p == 0 ? 20 : (p == 1 ? 8 : 0); }
struct SelCtx {
    unsigned int prefix_hi;  // the chosen prefix in place (key bits above the bins)
    unsigned int hi_mask;    // the bits it covers (0 in the first pass)
    int bin_shift;
    unsigned int bin_mask;
    int shift, base;    // LDS addressing as in Hist
    unsigned int *lds;
    unsigned int *s_cnt;     // candidates this block copied (LDS counter)
    float *cand;             // this block's candidate region
    unsigned int cand_cap;
};

// With COLLECT, every voxel that matches the prefix is also copied to the
// block's candidate region: one LDS atomic per wavefront step that has any
// match, each matching lane at its rank among the matches (mbcnt).
template <int NV, bool COLLECT = false>
__device__ __forceinline__ void select_step(const float (&x)[NV], unsigned long long &valid,
                                            const SelCtx &c)
{
    unsigned int cv = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const float v = x[j];
        const unsigned long long mv = __builtin_amdgcn_ballot_w64(v == v);
        cv += __popcll(mv);
        const unsigned int k = order_key(v);
        const bool match = ((k ^ c.prefix_hi) & c.hi_mask) == 0u;
        const unsigned long long inr = mv & __builtin_amdgcn_ballot_w64(match);
        const int b = (int)((k >> c.bin_shift) & c.bin_mask);
        // Only lanes whose voxel is valid and under the prefix count: after
        // the first pass most lanes do not, and sending them all to one
        // dummy slot would serialize the atomic on a few LDS words.
        if (v == v && match)
            atomicAdd((unsigned int *)((char *)c.lds + ((b << c.shift) + c.base)), 1u);
        if (COLLECT && inr) {  // wavefront-uniform
            const int lane = threadIdx.x & 63;
            unsigned int base = 0;
            if (lane == 0) base = atomicAdd(c.s_cnt, (unsigned int)__popcll(inr));
            base = __shfl(base, 0);
            if ((inr >> lane) & 1ull) {
                const unsigned int i =
                    base + __builtin_amdgcn_mbcnt_hi((unsigned int)(inr >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned int)inr, 0u));
                if (i < c.cand_cap) c.cand[i] = v;
            }
        }
    }
    asm("" : "+s"(cv));
    valid += cv;
}

// Counting step of a select pass (and, with COLLECT, copying).
template <bool COLLECT>
struct CountStep {
    SelCtx c;
    unsigned long long valid;
    template <int NV>
    __device__ __forceinline__ void operator()(const float (&x)[NV])
    {
        select_step<NV, COLLECT>(x, valid, c);
    }
};

// The smallest order key above K among valid voxels (per lane).
struct NextStep {
    unsigned int K, m;
    template <int NV>
    __device__ __forceinline__ void operator()(const float (&x)[NV])
    {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const unsigned int k = order_key(x[j]);
            m = (x[j] == x[j] && k > K && k < m) ? k : m;
        }
    }
};

__global__ void __launch_bounds__(1024) k_select(SelectArgs a)
{
    extern __shared__ unsigned int lds[];
    __shared__ unsigned int s_last, s_cnt;
    __shared__ int s_t;
    __shared__ unsigned long long s_rank;
    __shared__ unsigned long long s_part[1024];
    const int tid = threadIdx.x, B = blockDim.x;
    const int p = a.pass;
    const int width = sel_width(p);
    const int nbins = 1 << width;
    CountStep<false> cs;
    SelCtx &c = cs.c;
    const int top = sel_shift(p) + width;   // first key bit above this pass's bins
    c.hi_mask = p == 0 ? 0u : (0xffffffffu << top);
    c.prefix_hi = p == 0 ? 0u : (a.st->prefix << top);
    c.bin_shift = sel_shift(p);
    c.bin_mask = (unsigned int)nbins - 1u;
    const int C = 1 << a.copies_log2;
    c.shift = a.copies_log2 + 2;
    c.base = (C + (tid & 63 & (C - 1))) * 4;
    c.lds = lds;
    c.s_cnt = &s_cnt;
    c.cand = a.cand + (size_t)blockIdx.x * a.cand_cap;
    c.cand_cap = a.cand_cap;
    if (tid == 0) s_cnt = 0u;
    lds_zero(lds, nbins, a.copies_log2);
    cs.valid = 0;
    const bool collect = p == 1 && a.st->collect;
    const bool from_cand = p == 2 && a.st->collect && !a.st->overflow;
    if (collect) {
        CountStep<true> cc;
        cc.c = c;
        cc.valid = 0;
        scan_box(a.g, cc, a.claim);
        __syncthreads();
        if (tid == 0) {
            a.cand_n[blockIdx.x] = min(s_cnt, a.cand_cap);
            if (s_cnt > a.cand_cap) atomicOr(&a.st->overflow, 1u);
        }
    } else if (from_cand) {
        // The third pass over this block's candidates only (all valid, all
        // in the first pass's bucket), in wavefront-uniform steps.
        const unsigned int n = a.cand_n[blockIdx.x];
        for (unsigned int i0 = 0; i0 < n; i0 += (unsigned int)B) {
            const unsigned int i = i0 + (unsigned int)tid;
            float xv[1] = {i < n ? c.cand[i] : qnan()};
            select_step<1>(xv, cs.valid, c);
        }
    } else {
        scan_box(a.g, cs, a.claim);
    }
    const unsigned long long valid = cs.valid;
    const int lane = tid & 63;
    // Flush bins (slot b + 1 holds bin b); the valid count goes with the
    // first pass.
    __syncthreads();
    for (int b = tid; b < nbins; b += B) {
        unsigned int sum = 0;
        for (int k = 0; k < C; ++k) sum += lds[((b + 1) << a.copies_log2) + k];
        if (sum) atomicAdd(&a.acc[b], (unsigned long long)sum);
    }
    if (p == 0 && lane == 0 && valid) atomicAdd(&a.st->n_valid, valid);
    if (!last_to_arrive(a.ticket, gridDim.x, &s_last)) return;

    // Last block: find the bin holding the rank (counts in bin order), then
    // return the accumulators to zero.
    const int per = (nbins + B - 1) / B;
    unsigned long long mine = 0;
    for (int k = 0; k < per; ++k) {
        const int b = tid * per + k;
        if (b < nbins) mine += a.acc[b];
    }
    s_part[tid] = mine;
    SelectState st;
    if (tid == 0) {
        st = *a.st;
        if (p == 0 && st.rank_mode == 1 && st.n_valid) {
            st.rank = (st.n_valid - 1) / 2;
            st.want_next = (st.n_valid % 2 == 0) ? 1u : 0u;
        }
        if (p == 0 && st.rank >= st.n_valid) st.error = 1u;
        if (p == 0 && st.want_next && st.rank + 1 >= st.n_valid) st.want_next = 0u;
        s_rank = st.rank;
        s_t = B - 1;
    }
    // Inclusive prefix sums of the threads' partial counts, then the first
    // thread whose sum passes the rank (the last one if none does).
    for (int off = 1; off < B; off <<= 1) {
        __syncthreads();
        const unsigned long long v = tid >= off ? s_part[tid - off] : 0ull;
        __syncthreads();
        s_part[tid] += v;
    }
    __syncthreads();
    {
        const unsigned long long r = s_rank;
        if (tid < B - 1 && s_part[tid] > r && (tid == 0 || s_part[tid - 1] <= r)) s_t = tid;
    }
    __syncthreads();
    if (tid == 0) {
        if (!st.error) {
            const int t = s_t;
            unsigned long long before = t > 0 ? s_part[t - 1] : 0ull;
            int b = t * per;
            while (b < nbins - 1 && before + a.acc[b] <= st.rank) before += a.acc[b++];
            const unsigned int up = st.prefix << width;
            st.prefix = up | (unsigned int)b;
            st.rank -= before;
            // The second pass copies this bucket out when it fits the
            // candidate regions; the third then reads only those.
            if (p == 0)
                st.collect = a.cand && a.acc[b] <= (unsigned long long)a.cand_cap * gridDim.x
                                 ? 1u : 0u;
            if (p == 2) {
                st.value = key_value(st.prefix);
                if (a.out) *a.out = st.value;
                if (st.want_next) {
                    // The next rank is this key again, the next non-empty
                    // key of this histogram, or (neither) the smallest key
                    // above this one anywhere: one more pass.
                    if (st.rank + 1 < a.acc[b]) {
                        st.value_next = st.value;
                    } else {
                        int nb = b + 1;
                        while (nb < nbins && a.acc[nb] == 0ull) ++nb;
                        if (nb < nbins)
                            st.value_next = key_value(up | (unsigned int)nb);
                        else
                            st.need_next = 1u;
                    }
                }
            }
        }
        *a.st = st;
    }
    __syncthreads();
    for (int b = tid; b < nbins; b += B) a.acc[b] = 0ull;
    if (tid == 0) {
        *a.ticket = 0u;
        if (a.claim.nc) *a.claim.ctr = 0u;
    }
}

// The voxel of the next rank when the last histogram did not hold it: the
// smallest valid key above the selected one.  Every block exits at once
// unless it is needed.
__global__ void __launch_bounds__(1024) k_select_next(SelectArgs a)
{
    __shared__ unsigned int s_last;
    const int tid = threadIdx.x;
    if (!a.st->need_next || a.st->error) return;
    NextStep ns;
    ns.K = a.st->prefix;
    ns.m = 0xffffffffu;
    scan_box(a.g, ns, a.claim);
    unsigned int m = ns.m;
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned int o = __shfl_xor(m, off);
        m = o < m ? o : m;
    }
    if ((tid & 63) == 0 && m != 0xffffffffu) atomicMin(&a.st->next_key, m);
    if (!last_to_arrive(a.ticket, gridDim.x, &s_last) || tid != 0) return;
    a.st->value_next = key_value(__hip_atomic_load(&a.st->next_key, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT));
    *a.ticket = 0u;
    if (a.claim.nc) *a.claim.ctr = 0u;
}

}  // namespace cube

using namespace cube;

namespace {

// Candidate regions: 2^24 floats (64 MiB) shared out among the blocks.
constexpr unsigned int CAND_TOTAL = 1u << 24;

struct SelectWorkspace {
    SelectState *st = nullptr;
    unsigned long long *acc = nullptr;
    unsigned int *ticket = nullptr;
    SelectState *h_st = nullptr;  // pinned
    float *cand = nullptr;
    unsigned int *cand_n = nullptr;
    int cand_blocks = 0;          // blocks the candidate regions were cut for
};

std::mutex g_smu;
SelectWorkspace g_sws[64];
bool g_sws_ready[64];

int select_ws(SelectWorkspace **out)
{
    int dev = 0;
    hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return fail(CUBE_EINVAL, "device index out of range");
    if (!g_sws_ready[dev]) {
        SelectWorkspace &w = g_sws[dev];
        hipError_t e;
        if ((e = hipMalloc(&w.st, sizeof(SelectState))) != hipSuccess ||
            (e = hipMalloc(&w.acc, 4096 * 8)) != hipSuccess ||
            (e = hipMalloc(&w.ticket, 256)) != hipSuccess ||
            (e = hipHostMalloc(&w.h_st, sizeof(SelectState))) != hipSuccess ||
            (e = hipMemset(w.acc, 0, 4096 * 8)) != hipSuccess ||
            (e = hipMemset(w.ticket, 0, 256)) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess)
            return hip_fail(e, "select workspace");
        g_sws_ready[dev] = true;
    }
    *out = &g_sws[dev];
    return CUBE_OK;
}

// Three passes on the default stream (and, for the median of an even count,
// at most one more); the result is read back.  The third pass reads only the
// candidates the second copied out, unless they did not fit.  With rank_mode 1 the rank is
// the lower middle of the valid voxels and, for an even count, *next is the
// upper middle.
int select_rank(const Box &b, uint64_t rank, int rank_mode, float *value, uint64_t *n_valid,
                float *next = nullptr)
{
    SelectWorkspace *w = nullptr;
    int rc = select_ws(&w);
    if (rc) return rc;
    SelectState init;
    memset(&init, 0, sizeof init);
    init.rank = rank;
    init.rank_mode = (unsigned int)rank_mode;
    init.next_key = 0xffffffffu;
    hipError_t e;
    // Synchronous copy: the workspace is reused by the next call.
    if ((e = hipMemcpy(w->st, &init, sizeof init, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "select state");
    SelectArgs a;
    memset(&a, 0, sizeof a);
    const int threads = 1024;
    const void *ksel = reinterpret_cast<const void *>(&k_select);
    // One grid for every pass (pass 2 reads the candidates of its own block
    // index), sized by the largest pass's LDS: 4096 bins in 8 copies.
    int blocks = 0, chunks = 0;
    if ((rc = scan_plan(b, ksel, threads, (size_t)(4096 + 2) * 8 * 4, &blocks, &chunks)))
        return rc;
    scan_geom(b, chunks > blocks ? chunks : blocks, &a.g);
    a.st = w->st;
    a.acc = w->acc;
    a.ticket = w->ticket;
    a.claim.ctr = w->ticket + CHUNK_CTR_WORD;
    a.claim.nc = chunks;
    if (w->cand_blocks < blocks) {
        hipFree(w->cand_n);
        w->cand_n = nullptr;
        w->cand_blocks = 0;
        if ((e = hipMalloc(&w->cand_n, (size_t)blocks * 4)) != hipSuccess)
            return hip_fail(e, "select candidates");
        w->cand_blocks = blocks;
    }
    if (!w->cand && (e = hipMalloc(&w->cand, (size_t)CAND_TOTAL * 4)) != hipSuccess)
        return hip_fail(e, "select candidates");
    a.cand = w->cand;
    a.cand_n = w->cand_n;
    a.cand_cap = CAND_TOTAL / (unsigned int)blocks;
    for (int p = 0; p < 3; ++p) {
        a.pass = p;
        const int nb = 1 << sel_width(p);
        a.copies_log2 = nb >= 4096 ? 3 : 5;
        const size_t lds = ((size_t)(nb + 2) << a.copies_log2) * 4;
        const void *k = reinterpret_cast<const void *>(&k_select);
        if (lds > 64 * 1024 &&
            (e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
                hipSuccess)
            return hip_fail(e, "select LDS");
        SelectArgs ac = a;
        void *args[] = {&ac};
        if ((e = hipLaunchKernel(k, dim3((unsigned)blocks), dim3(threads), args, lds, nullptr)) !=
            hipSuccess)
            return hip_fail(e, "select launch");
    }
    if (rank_mode == 1) {
        SelectArgs ac = a;
        void *args[] = {&ac};
        if ((e = hipLaunchKernel(reinterpret_cast<const void *>(&k_select_next),
                                 dim3((unsigned)blocks), dim3(threads), args, 0, nullptr)) !=
            hipSuccess)
            return hip_fail(e, "select launch");
    }
    if ((e = hipMemcpy(w->h_st, w->st, sizeof(SelectState), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "select result");
    if (n_valid) *n_valid = w->h_st->n_valid;
    if (w->h_st->error)
        return fail(CUBE_EINVAL, "rank %llu >= %llu valid voxels", (unsigned long long)rank,
                    (unsigned long long)w->h_st->n_valid);
    *value = w->h_st->value;
    if (next) *next = w->h_st->want_next ? w->h_st->value_next : w->h_st->value;
    return CUBE_OK;
}

}  // namespace

extern "C" {

int cube_select(const float *ptr, const int64_t *dims, uint64_t rank, float *value)
{
    CUBE_GUARD_BEGIN
    if (!value) return fail(CUBE_EINVAL, "value is NULL");
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (!rc) rc = check_box_device(&b);
    if (rc) return rc;
    if (b.n == 0) return fail(CUBE_EINVAL, "empty box");
    std::lock_guard<std::mutex> lk(g_smu);
    return select_rank(b, rank, 0, value, nullptr);
    CUBE_GUARD_END
}

int cube_median(const float *ptr, const int64_t *dims, double *median, uint64_t *n_valid)
{
    CUBE_GUARD_BEGIN
    if (!median) return fail(CUBE_EINVAL, "median is NULL");
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (!rc) rc = check_box_device(&b);
    if (rc) return rc;
    if (b.n == 0) return fail(CUBE_EINVAL, "empty box");
    std::lock_guard<std::mutex> lk(g_smu);
    // The lower middle (which is the median for odd n_valid), then for even
    // n_valid the upper middle too.
    float a = 0.f, c = 0.f;
    uint64_t n = 0;
    rc = select_rank(b, 0, 1, &a, &n, &c);
    if (n_valid) *n_valid = n;
    if (n == 0) return fail(CUBE_EINVAL, "no valid voxel");
    if (rc) return rc;
    *median = n % 2 == 1 ? (double)a : ((double)a + (double)c) / 2.0;
    return CUBE_OK;
    CUBE_GUARD_END
}

}  // extern "C"
