// Host side of libpbit: argument checks, the workspace plan, and the C ABI
// declared in include/pbit.h.  All device work is queued by enqueue_sort().
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "pbit.h"
#include "pbit_internal.h"

namespace pbit {

hipError_t enqueue_sort(const Plan& P, uint32_t head, const uint32_t* next_in, uint32_t* next_out,
                        const void* keys, uint32_t* d_result, char* ws, hipStream_t s, Prof* prof);
hipError_t enqueue_empty(uint32_t* d_result, hipStream_t s);
hipError_t enqueue_sort_aos(const Plan& P, uint32_t head, char* base, uint64_t stride,
                            uint32_t next_off, uint32_t key_off, uint32_t* d_result, char* ws,
                            hipStream_t s, Prof* prof);
hipError_t enqueue_sort_lists(const Plan& P, const uint32_t* heads, const uint64_t* offsets,
                              const uint32_t* next_in, uint32_t* next_out, const void* keys,
                              const uint64_t* next_in_ptrs, const uint64_t* next_out_ptrs,
                              const uint64_t* key_ptrs, uint32_t* new_heads, int32_t* d_status,
                              char* ws, hipStream_t s, Prof* prof);
hipError_t enqueue_repair_prev(const uint32_t* heads, uint32_t num_lists, const uint32_t* next,
                               uint32_t* prev, uint32_t n, int32_t* status, hipStream_t s);
uint32_t pass_tile(uint32_t key_bytes, uint32_t rb);

// Look-back spin bound given to every digit pass queued from now on.
static std::atomic<uint32_t> g_spin_limit{kSpinLimit};

static size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

static size_t entry_bytes(uint32_t key_bytes) { return key_bytes == 8 ? 16 : 8; }
static size_t node_bytes(uint32_t key_bytes) { return key_bytes == 8 ? 16 : 8; }
static size_t pair_bytes(uint32_t key_bytes) { return key_bytes == 8 ? 12 : 8; }
// Entries a level-0 walker gathers in registers per burst (the device SegLen).
static uint32_t reg_entries(uint32_t key_bytes)
{
    return key_bytes == 8 ? PBIT_SEGLEN / 2 : PBIT_SEGLEN;
}

// Entries stored per level-0 chain (a multiple of the walker's register
// block).  Chain lengths are geometric with mean 16, so a slot of 128 leaves
// about 1 chain in 4000 with a rest to re-walk and 64 about 1 in 60; the slots
// cost 8 (16 for 64-bit keys) bytes per entry, so larger inputs get less.
static uint32_t level0_cap(uint64_t n, uint32_t reg)
{
    if (n <= (1ull << 26))
        return 128u;
    if (n <= (1ull << 31))
        return 64u > reg ? 64u : reg;
    return reg;
}

// ---------------------------------------------------------------- tuning
// Choices the caller leaves to the library (K = 0; the short-list cutoff of
// many-list sorts).  An entry applies to sorts of its kind (0: one list, 1:
// many lists) and key width whose node count is at most n_max; the first
// such entry in order of n_max wins.  The built-in table comes from device
// measurements (pbit_tuning.h, written by the package's tuner);
// pbit_tune_set adds or replaces entries at run time.
struct TuneEntry {
    uint32_t kind, M;
    uint64_t n_max;
    uint32_t K, cutoff;
};
#include "pbit_tuning.h"

constexpr int kMaxTune = 128;
static std::mutex g_tune_mu;
static TuneEntry g_tune[kMaxTune];
static int g_ntune = -1;  // -1: the built-in table not yet loaded

static void tune_init_locked()
{
    if (g_ntune >= 0)
        return;
    g_ntune = 0;
    for (const TuneEntry& t : kBuiltinTuning)
        if (g_ntune < kMaxTune)
            g_tune[g_ntune++] = t;
}

static bool valid_cutoff(uint32_t c) { return c == 1024 || c == 2048 || c == 4096; }

// K (when 0 is passed) and the cutoff for a sort of this kind, width and size.
static void tune_lookup(uint32_t kind, uint32_t M, uint64_t n, uint32_t* K, uint32_t* cutoff)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_init_locked();
    const TuneEntry* best = nullptr;
    for (int i = 0; i < g_ntune; i++) {
        const TuneEntry& t = g_tune[i];
        if (t.kind == kind && t.M == M && n <= t.n_max && (!best || t.n_max < best->n_max))
            best = &t;
    }
    *K = best ? best->K : (M == 8 ? 4u : 8u);
    *cutoff = best ? best->cutoff : 2048u;
}

static bool valid_k(uint32_t M, uint32_t K)
{
    if (M != 8 && M != 16 && M != 32 && M != 64)
        return false;
    if (K != 1 && K != 2 && K != 4 && K != 8)
        return false;
    return (M % K) == 0;
}

static bool valid_shape(uint32_t M, uint32_t K)
{
    if (M != 8 && M != 16 && M != 32 && M != 64)
        return false;
    return K == 0 || valid_k(M, K);
}

// Regions every sort uses: header, histograms, look-back words (and, for
// many lists, the per-segment digit counts: the zeroed region ends there),
// packed nodes, the two list-order buffers and the level-0 chain arrays.
// K is resolved (not 0).
static bool plan_common(uint64_t n, uint32_t M, uint32_t K, uint32_t flags, size_t lw_bytes,
                        uint64_t level0_chains, uint32_t cap, size_t lcnt_bytes, Plan* P,
                        size_t& off)
{
    if (!valid_k(M, K) ||
        (flags & ~(uint32_t)(PBIT_DESCENDING | PBIT_SIGNED | PBIT_FLOAT | PBIT_SHARED)) != 0 ||
        ((flags & PBIT_SIGNED) && (flags & PBIT_FLOAT)))
        return false;
    P->n = n;
    P->M = M;
    P->K = K;
    P->RB = P->K;
    P->radix = 1u << P->K;
    P->passes = M / P->K;
    if (P->passes > (uint32_t)kMaxPasses)
        return false;
    P->flags = flags;
    P->look64 = lw_bytes == 8;
    P->spin_limit = g_spin_limit.load(std::memory_order_relaxed);
    P->key_bytes = M / 8;
    P->tile = pass_tile(P->key_bytes, P->RB);
    P->tiles = (uint32_t)ceil_div(n ? n : 1, P->tile);
    // the passes over the high half of one list's 64-bit keys (set by the
    // single-list planner) use the 32-bit shape
    P->hi_from = P->passes;
    P->tiles_hi = (uint32_t)ceil_div(n ? n : 1, pass_tile(4, P->RB));
    P->look_tiles = P->key_bytes == 8 ? (P->tiles > P->tiles_hi ? P->tiles : P->tiles_hi) : P->tiles;
    off = 0;
    P->o_header = off;
    off = align_up(off + sizeof(Header));
    P->o_hist = off;
    off = align_up(off + (size_t)P->passes * P->radix * 4);
    P->o_dbase = off;
    off = align_up(off + (size_t)P->passes * P->radix * 4);
    P->o_look = off;
    off = align_up(off + (size_t)P->passes * P->look_tiles * P->radix * lw_bytes);
    P->o_lcnt = off;
    off = align_up(off + lcnt_bytes);
    P->zero_end = off;
    P->o_nodes = off;
    off = align_up(off + n * node_bytes(P->key_bytes));
    P->o_pairsA = off;
    off = align_up(off + n * pair_bytes(P->key_bytes));
    P->o_pairsB = off;
    off = align_up(off + n * pair_bytes(P->key_bytes));
    P->o_idxA = off;
    off = align_up(off + n * 4);
    P->o_idxB = P->o_idxA;  // node indices are written once, by the last pass
    LevelPlan& L = P->lv[0];
    L.log_l = kLog0;
    L.m = n;
    L.n_static = level0_chains;
    L.cap = cap;
    L.o_chain_rec = off;
    off = align_up(off + L.n_static * 8);
    L.o_ent = off;
    off = align_up(off + L.n_static * cap * entry_bytes(P->key_bytes));
    L.o_resume = off;
    off = align_up(off + L.n_static * 4);
    L.o_long = off;
    off = align_up(off + (size_t)2 * kLongListMax * 4);
    L.o_offn = off;
    off = align_up(off + L.n_static * 4);
    return true;
}

// Workspace layout for one list.  Returns false on arguments the C ABI rejects.
bool make_plan(uint64_t n, uint32_t M, uint32_t K, uint32_t flags, Plan* P)
{
    memset(P, 0, sizeof(*P));
    if (n > PBIT_MAX_NODES || !valid_shape(M, K))
        return false;
    // the table gives K (when 0 is passed) and the size up to which one
    // workgroup sorts the whole list in LDS
    uint32_t tuned_k, cut;
    tune_lookup(0, M, n, &tuned_k, &cut);
    if (K == 0)
        K = tuned_k;
    if (n == 0) {
        size_t off;
        if (!plan_common(0, M, K, flags, 4, 0, 0, 0, P, off))
            return false;
        P->total = 256;
        return true;
    }
    const uint32_t reg = reg_entries(M / 8);
    const uint32_t cap = level0_cap(n, reg);
    // a look-back word holds a 30-bit count next to its 2 flag bits; from
    // 2^30 nodes on the words are 64 bits wide
    const size_t lw_bytes = n >= (1ull << 30) ? 8 : 4;
    size_t off = 0;
    if (!plan_common(n, M, K, flags, lw_bytes, 1 + ceil_div(n, 1ull << kLog0), cap, 0, P, off))
        return false;
    if (P->key_bytes == 8)
        P->hi_from = P->passes / 2;
    int k = 1;
    uint64_t m = P->lv[0].n_static;
    while (m > kBaseMax) {
        if (k >= kMaxLevels)
            return false;
        LevelPlan& L = P->lv[k];
        L.log_l = kLogUp;
        L.m = m;
        L.n_static = 1 + ceil_div(m, 1ull << L.log_l);
        L.o_chain_rec = off;
        off = align_up(off + L.n_static * 8);
        L.o_offn = off;
        off = align_up(off + L.n_static * 4);
        m = L.n_static;
        k++;
    }
    P->levels = k;
    // relink through node ranges held in LDS (see k_relink_ranges)
    if (n >= kRelinkMinNodes && n <= kRelinkMaxNodes) {
        P->relink_r = n <= (uint64_t)kRelinkRangesMax << 14 ? 14u : 15u;
        P->relink_ranges = (uint32_t)ceil_div(n, 1ull << P->relink_r);
        P->relink_tiles = (uint32_t)ceil_div(n, kRelinkTile);
        P->o_rstart = off;
        off = align_up(off + (size_t)(P->relink_ranges + 1) * P->relink_tiles * 4);
    }
    P->total = off;
    P->cutoff = valid_cutoff(cut) ? cut : 0u;
    return true;
}

// Workspace layout for num_lists lists over n nodes in total.  The regions
// that depend on how many lists exceed the cutoff are sized for the smallest
// cutoff (kMinSegLen), so a workspace stays large enough whatever cutoff the
// tuning table gives later.
bool make_plan_lists(uint64_t n, uint32_t num_lists, uint32_t M, uint32_t K, uint32_t flags,
                     Plan* P)
{
    memset(P, 0, sizeof(*P));
    // one workgroup per list sorts the short ones: the list count is a grid size
    if (num_lists == 0 || num_lists > 0x7FFFFFFFu || n >= (uint64_t)PBIT_NIL ||
        !valid_shape(M, K))
        return false;
    uint32_t Kt, cutoff;
    tune_lookup(1, M, n, &Kt, &cutoff);
    if (K == 0)
        K = Kt;
    if (!valid_k(M, K) || !valid_cutoff(cutoff))
        return false;
    const uint32_t reg = reg_entries(M / 8);
    const uint32_t cap = level0_cap(n, reg);
    const uint64_t chains0 = (uint64_t)num_lists + ceil_div(n, 1ull << kLog0);
    if (chains0 >= (uint64_t)PBIT_NIL)
        return false;
    uint64_t seg_max = n / (kMinSegLen + 1);
    if (seg_max > num_lists)
        seg_max = num_lists;
    if (seg_max == 0)
        seg_max = 1;
    const uint64_t seg_chunks = ceil_div(seg_max, kSegChunk);
    const uint32_t passes = M / K, radix = 1u << K;
    const size_t lcnt_bytes = (size_t)passes * seg_max * radix * 4;
    const size_t lw_bytes = n >= (1ull << 30) ? 8 : 4;
    size_t off = 0;
    if (!plan_common(n, M, K, flags, lw_bytes, chains0, cap, lcnt_bytes, P, off))
        return false;
    P->num_lists = num_lists;
    P->log_block = 8;
    P->cutoff = cutoff;
    P->seg_max = (uint32_t)seg_max;
    P->seg_chunks = (uint32_t)seg_chunks;
    // nodes per pack block: its digit counts flush once per block, so large
    // chunks (whole steps of 4 waves x 256 nodes)
    P->pack_chunk = 32768;
    P->o_table = off;
    off = align_up(off + (ceil_div(n, 1ull << P->log_block) + 1) * 4);
    P->o_headbits = off;  // cleared by its own launch at the start of every sort
    off = align_up(off + (ceil_div(n, 32) + 1) * 4);
    P->o_lseg = off;
    off = align_up(off + ((size_t)num_lists + 1) * 4);
    P->o_segl = off;
    off = align_up(off + seg_max * 4);
    P->o_coff = off;
    off = align_up(off + (seg_max + 1) * 4);
    P->o_ctable = off;
    off = align_up(off + (ceil_div(n, 1ull << kSegLog) + 1) * 4);
    P->o_lbase = off;
    off = align_up(off + lcnt_bytes);
    P->o_csum = off;
    off = align_up(off + (size_t)passes * seg_chunks * radix * 4);
    P->o_snext = off;
    off = align_up(off + n * 4);
    P->o_shead = off;
    off = align_up(off + (size_t)num_lists * 4);
    int lv = 1;
    uint64_t m = chains0;
    while (m > num_lists) {
        if (lv >= kMaxLevels)
            return false;
        LevelPlan& L = P->lv[lv];
        L.log_l = 3;
        L.m = m;
        L.n_static = num_lists + (m - num_lists) / 8;
        L.o_chain_rec = off;
        off = align_up(off + L.n_static * 8);
        L.o_offn = off;
        off = align_up(off + L.n_static * 4);
        m = L.n_static;
        lv++;
    }
    P->levels = lv;
    P->total = off;
    return true;
}

struct SyncCache {
    std::mutex mu;
    void* ws = nullptr;
    size_t bytes = 0;
    uint32_t* result = nullptr;
};

static SyncCache& sync_cache(int dev)
{
    static SyncCache caches[64];
    return caches[dev & 63];
}

}  // namespace pbit

using namespace pbit;

extern "C" size_t pbit_workspace_bytes(uint64_t n, uint32_t M, uint32_t K)
{
    Plan P;
    if (!make_plan(n, M, K, 0, &P))
        return 0;
    return P.total;
}

static int sort_list_async_impl(uint32_t head, const uint32_t* next_in, uint32_t* next_out,
                                const void* keys, uint64_t n, uint32_t M, uint32_t K,
                                uint32_t flags, uint32_t* d_result, void* ws, size_t ws_bytes,
                                void* stream, Prof* prof)
{
    hipStream_t s = (hipStream_t)stream;
    if (!d_result || ((uintptr_t)d_result & 3u))
        return PBIT_EINVAL;
    Plan P;
    if (!make_plan(n, M, K, flags, &P))
        return PBIT_EINVAL;
    if (n == 0) {
        if (head != PBIT_NIL)
            return PBIT_EINVAL;
        return enqueue_empty(d_result, s) == hipSuccess ? PBIT_OK : PBIT_EHIP;
    }
    if (head >= n)
        return PBIT_EINVAL;
    if (!next_in || !next_out || !keys || !ws)
        return PBIT_EINVAL;
    if (((uintptr_t)next_in & 3u) || ((uintptr_t)next_out & 3u) ||
        ((uintptr_t)keys & (P.key_bytes - 1)) || ((uintptr_t)ws & 255u))
        return PBIT_EINVAL;
    if (ws_bytes < P.total)
        return PBIT_ENOMEM;
    hipError_t e = enqueue_sort(P, head, next_in, next_out, keys, d_result, (char*)ws, s, prof);
    return e == hipSuccess ? PBIT_OK : PBIT_EHIP;
}

extern "C" int pbit_sort_list_async(uint32_t head, const uint32_t* next_in, uint32_t* next_out,
                                    const void* keys, uint64_t n, uint32_t M, uint32_t K,
                                    uint32_t flags, uint32_t* d_result, void* ws,
                                    size_t ws_bytes, void* stream)
{
    return sort_list_async_impl(head, next_in, next_out, keys, n, M, K, flags, d_result, ws,
                                ws_bytes, stream, nullptr);
}

// ---------------------------------------------------------------- no allocation
// Workspace of pbit_sort_list_noalloc: one array in every device's memory for
// the life of the process.  Host code never passes `scratch` itself to a
// kernel (on the host it names a stand-in, not device memory): the device
// address of each device's copy is looked up once per device and kept.
static __device__ __align__(256) unsigned char scratch[PBIT_NOALLOC_SCRATCH_BYTES];

struct ScratchSlot {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};

static ScratchSlot& scratch_slot(int dev)
{
    static ScratchSlot slots[64];
    return slots[dev & 63];
}

// Device address of the current device's scratch array (nullptr on failure).
static void* scratch_ptr()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    ScratchSlot& sl = scratch_slot(dev);
    std::call_once(sl.once, [&sl]() {
        void* p = nullptr;
        sl.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        sl.ptr = sl.err == hipSuccess ? p : nullptr;
    });
    return sl.ptr;
}

extern "C" int pbit_sort_list_noalloc(uint32_t head, const uint32_t* next_in, uint32_t* next_out,
                                      const void* keys, uint64_t n, uint32_t M, uint32_t K,
                                      uint32_t flags, uint32_t* d_result, void* stream)
{
    Plan P;
    if (!make_plan(n, M, K, flags, &P))
        return PBIT_EINVAL;
    if (P.total > (size_t)PBIT_NOALLOC_SCRATCH_BYTES)
        return PBIT_ENOMEM;  // the list needs more workspace than the fixed array holds
    void* ws = scratch_ptr();
    if (!ws)
        return PBIT_EHIP;
    // the same kernels as pbit_sort_list_async, on the fixed array; every
    // region that must start at zero is cleared by the sort's own first
    // kernel, so nothing left by an earlier call matters
    return sort_list_async_impl(head, next_in, next_out, keys, n, M, K, flags, d_result, ws,
                                (size_t)PBIT_NOALLOC_SCRATCH_BYTES, stream, nullptr);
}

extern "C" int pbit_sort_list_profiled(uint32_t head, const uint32_t* next_in,
                                       uint32_t* next_out, const void* keys, uint64_t n,
                                       uint32_t M, uint32_t K, uint32_t flags,
                                       uint32_t* d_result, void* ws, size_t ws_bytes,
                                       void* stream, void** events, int32_t* stage_ids,
                                       int n_events, int* n_recorded)
{
    if (!events || n_events <= 0 || !n_recorded)
        return PBIT_EINVAL;
    Prof prof{events, stage_ids, n_events, 0};
    int st = sort_list_async_impl(head, next_in, next_out, keys, n, M, K, flags, d_result, ws,
                                  ws_bytes, stream, &prof);
    *n_recorded = prof.count;
    return st;
}

extern "C" int pbit_sort_list_aos_async(uint32_t head, void* nodes, uint64_t stride,
                                        uint32_t next_off, uint32_t key_off, uint64_t n,
                                        uint32_t M, uint32_t K, uint32_t flags,
                                        uint32_t* d_result, void* ws, size_t ws_bytes,
                                        void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (!d_result || ((uintptr_t)d_result & 3u))
        return PBIT_EINVAL;
    Plan P;
    if (!make_plan(n, M, K, flags, &P))
        return PBIT_EINVAL;
    if (n == 0) {
        if (head != PBIT_NIL)
            return PBIT_EINVAL;
        return enqueue_empty(d_result, s) == hipSuccess ? PBIT_OK : PBIT_EHIP;
    }
    const uint64_t kb = P.key_bytes;
    const uintptr_t base = (uintptr_t)nodes;
    if (head >= n || !nodes || !ws)
        return PBIT_EINVAL;
    // both fields inside the record, apart, and naturally aligned in every record
    if (stride < 4 || stride >= (1ull << 32) || (stride & 3u) || (stride % kb) != 0)
        return PBIT_EINVAL;
    if ((uint64_t)next_off + 4 > stride || (uint64_t)key_off + kb > stride)
        return PBIT_EINVAL;
    if (!((uint64_t)next_off + 4 <= key_off || (uint64_t)key_off + kb <= next_off))
        return PBIT_EINVAL;
    if (((base + next_off) & 3u) || ((base + key_off) & (kb - 1)) || ((uintptr_t)ws & 255u))
        return PBIT_EINVAL;
    if (ws_bytes < P.total)
        return PBIT_ENOMEM;
    hipError_t e = enqueue_sort_aos(P, head, (char*)nodes, stride, next_off, key_off, d_result,
                                    (char*)ws, s, nullptr);
    return e == hipSuccess ? PBIT_OK : PBIT_EHIP;
}

extern "C" int pbit_repair_prev_async(const uint32_t* d_heads, uint32_t num_lists,
                                      const uint32_t* next, uint32_t* prev, uint64_t n,
                                      int32_t* d_status, void* stream)
{
    if (n >= (uint64_t)PBIT_NIL)
        return PBIT_EINVAL;
    if (n == 0 && num_lists == 0)
        return PBIT_OK;
    if (num_lists && !d_heads)
        return PBIT_EINVAL;
    if (n && (!next || !prev))
        return PBIT_EINVAL;
    if (next && prev && (const void*)next == (const void*)prev)
        return PBIT_EINVAL;
    if (((uintptr_t)d_heads & 3u) || ((uintptr_t)next & 3u) || ((uintptr_t)prev & 3u) ||
        ((uintptr_t)d_status & 3u))
        return PBIT_EINVAL;
    hipError_t e = enqueue_repair_prev(d_heads, num_lists, next, prev, (uint32_t)n, d_status,
                                       (hipStream_t)stream);
    return e == hipSuccess ? PBIT_OK : PBIT_EHIP;
}

extern "C" const char* pbit_stage_name(int stage)
{
    static const char* names[] = {"zero", "pack", "walk0", "walk_up", "base", "down",
                                  "unchain", "schedule", "digit_pass", "relink", "plan",
                                  "small_lists", "bases", "commit", "end"};
    static_assert(sizeof(names) / sizeof(names[0]) == kStageCount + 1, "stage names");
    if (stage < 0 || stage > (int)kStageCount)
        return "unknown";
    return names[stage];
}

extern "C" int64_t pbit_sort_list(uint32_t head, uint32_t* next, const void* keys, uint64_t n,
                                  uint32_t M, uint32_t K)
{
    Plan P;
    if (!make_plan(n, M, K, 0, &P))
        return PBIT_EINVAL;
    if (n == 0)
        return head == PBIT_NIL ? (int64_t)PBIT_NIL : PBIT_EINVAL;
    if (head >= n || !next || !keys)
        return PBIT_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return PBIT_EHIP;
    SyncCache& c = sync_cache(dev);
    std::lock_guard<std::mutex> lock(c.mu);
    if (!c.result) {
        if (hipMalloc((void**)&c.result, 256) != hipSuccess)
            return PBIT_EHIP;
    }
    if (c.bytes < P.total) {
        if (c.ws) {
            if (hipDeviceSynchronize() != hipSuccess)
                return PBIT_EHIP;
            (void)hipFree(c.ws);
            c.ws = nullptr;
            c.bytes = 0;
        }
        if (hipMalloc(&c.ws, P.total) != hipSuccess)
            return PBIT_ENOMEM;
        c.bytes = P.total;
    }
    int st = pbit_sort_list_async(head, next, next, keys, n, M, K, 0, c.result, c.ws, c.bytes,
                                  nullptr);
    if (st != PBIT_OK)
        return st;
    uint32_t res[2];
    if (hipMemcpy(res, c.result, sizeof res, hipMemcpyDeviceToHost) != hipSuccess)
        return PBIT_EHIP;
    if ((int32_t)res[1] != 0)
        return (int32_t)res[1];
    return (int64_t)res[0];
}

extern "C" size_t pbit_lists_workspace_bytes(uint64_t total_nodes, uint32_t num_lists, uint32_t M,
                                             uint32_t K)
{
    Plan P;
    if (!make_plan_lists(total_nodes, num_lists, M, K, 0, &P))
        return 0;
    return P.total;
}

static int sort_lists_impl(const uint32_t* d_heads, const uint64_t* d_offsets, uint32_t num_lists,
                           uint64_t total_nodes, const uint32_t* next_in, uint32_t* next_out,
                           const void* keys, uint32_t M, uint32_t K, uint32_t flags,
                           uint32_t* d_new_heads, int32_t* d_status, void* ws, size_t ws_bytes,
                           void* stream, Prof* prof)
{
    Plan P;
    if (!make_plan_lists(total_nodes, num_lists, M, K, flags, &P))
        return PBIT_EINVAL;
    if (!d_heads || !d_offsets || !d_new_heads || !d_status || !ws)
        return PBIT_EINVAL;
    if (total_nodes > 0 && (!next_in || !next_out || !keys))
        return PBIT_EINVAL;
    if (((uintptr_t)d_heads & 3u) || ((uintptr_t)d_offsets & 7u) || ((uintptr_t)d_new_heads & 3u) ||
        ((uintptr_t)d_status & 3u) || ((uintptr_t)next_in & 3u) || ((uintptr_t)next_out & 3u) ||
        ((uintptr_t)keys & (P.key_bytes - 1)) || ((uintptr_t)ws & 255u))
        return PBIT_EINVAL;
    if (ws_bytes < P.total)
        return PBIT_ENOMEM;
    hipError_t e = enqueue_sort_lists(P, d_heads, d_offsets, next_in, next_out, keys, nullptr,
                                      nullptr, nullptr, d_new_heads, d_status, (char*)ws,
                                      (hipStream_t)stream, prof);
    return e == hipSuccess ? PBIT_OK : PBIT_EHIP;
}

extern "C" int pbit_sort_lists_gather(const uint32_t* d_heads, const uint64_t* d_offsets,
                                      uint32_t num_lists, uint64_t total_nodes,
                                      const uint64_t* d_next_in_ptrs,
                                      const uint64_t* d_next_out_ptrs,
                                      const uint64_t* d_key_ptrs, uint32_t M, uint32_t K,
                                      uint32_t flags, uint32_t* d_new_heads, int32_t* d_status,
                                      void* ws, size_t ws_bytes, void* stream)
{
    Plan P;
    if (!make_plan_lists(total_nodes, num_lists, M, K, flags, &P))
        return PBIT_EINVAL;
    if (!d_heads || !d_offsets || !d_new_heads || !d_status || !ws || !d_next_in_ptrs ||
        !d_next_out_ptrs || !d_key_ptrs)
        return PBIT_EINVAL;
    if (((uintptr_t)d_heads & 3u) || ((uintptr_t)d_offsets & 7u) || ((uintptr_t)d_new_heads & 3u) ||
        ((uintptr_t)d_status & 3u) || ((uintptr_t)d_next_in_ptrs & 7u) ||
        ((uintptr_t)d_next_out_ptrs & 7u) || ((uintptr_t)d_key_ptrs & 7u) ||
        ((uintptr_t)ws & 255u))
        return PBIT_EINVAL;
    if (ws_bytes < P.total)
        return PBIT_ENOMEM;
    hipError_t e = enqueue_sort_lists(P, d_heads, d_offsets, nullptr, nullptr, nullptr,
                                      d_next_in_ptrs, d_next_out_ptrs, d_key_ptrs, d_new_heads,
                                      d_status, (char*)ws, (hipStream_t)stream, nullptr);
    return e == hipSuccess ? PBIT_OK : PBIT_EHIP;
}

extern "C" int pbit_sort_lists(const uint32_t* d_heads, const uint64_t* d_offsets,
                               uint32_t num_lists, uint64_t total_nodes, const uint32_t* next_in,
                               uint32_t* next_out, const void* keys, uint32_t M, uint32_t K,
                               uint32_t flags, uint32_t* d_new_heads, int32_t* d_status, void* ws,
                               size_t ws_bytes, void* stream)
{
    return sort_lists_impl(d_heads, d_offsets, num_lists, total_nodes, next_in, next_out, keys, M,
                           K, flags, d_new_heads, d_status, ws, ws_bytes, stream, nullptr);
}

extern "C" int pbit_sort_lists_profiled(const uint32_t* d_heads, const uint64_t* d_offsets,
                                        uint32_t num_lists, uint64_t total_nodes,
                                        const uint32_t* next_in, uint32_t* next_out,
                                        const void* keys, uint32_t M, uint32_t K, uint32_t flags,
                                        uint32_t* d_new_heads, int32_t* d_status, void* ws,
                                        size_t ws_bytes, void* stream, void** events,
                                        int32_t* stage_ids, int n_events, int* n_recorded)
{
    if (!events || n_events <= 0 || !n_recorded)
        return PBIT_EINVAL;
    Prof prof{events, stage_ids, n_events, 0};
    const int st = sort_lists_impl(d_heads, d_offsets, num_lists, total_nodes, next_in, next_out,
                                   keys, M, K, flags, d_new_heads, d_status, ws, ws_bytes, stream,
                                   &prof);
    *n_recorded = prof.count;
    return st;
}

extern "C" int pbit_tune_set(uint32_t kind, uint32_t M, uint64_t n_max, uint32_t K,
                             uint32_t cutoff)
{
    if (kind > 1 || !valid_k(M, K) || !valid_cutoff(cutoff))
        return PBIT_EINVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_init_locked();
    for (int i = 0; i < g_ntune; i++) {
        TuneEntry& t = g_tune[i];
        if (t.kind == kind && t.M == M && t.n_max == n_max) {
            t.K = K;
            t.cutoff = cutoff;
            return PBIT_OK;
        }
    }
    if (g_ntune >= kMaxTune)
        return PBIT_ENOMEM;
    g_tune[g_ntune++] = TuneEntry{kind, M, n_max, K, cutoff};
    return PBIT_OK;
}

extern "C" void pbit_tune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_ntune = 0;
}

extern "C" void pbit_tune_reset(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_ntune = -1;
    tune_init_locked();
}

extern "C" int pbit_tune_lookup(uint32_t kind, uint32_t M, uint64_t n, uint32_t* K,
                                uint32_t* cutoff)
{
    if (kind > 1 || !K || !cutoff || !valid_shape(M, 0))
        return PBIT_EINVAL;
    tune_lookup(kind, M, n, K, cutoff);
    return PBIT_OK;
}

extern "C" uint32_t pbit_set_lookback_spin_limit(uint32_t sleeps)
{
    return g_spin_limit.exchange(sleeps, std::memory_order_relaxed);
}

extern "C" const char* pbit_status_string(int code)
{
    switch (code) {
    case PBIT_OK: return "ok";
    case PBIT_EINVAL: return "invalid argument";
    case PBIT_EMALFORMED: return "malformed list (index out of range, cycle, or length != n)";
    case PBIT_ENOMEM: return "workspace too small";
    case PBIT_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

extern "C" const char* pbit_version(void)
{
    return "pbit-mi355x 0.1 (gfx950)";
}
