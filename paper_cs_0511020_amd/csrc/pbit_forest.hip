// Many independent lists sorted together (HIP, gfx950).
//
// List l owns the node slab [offsets[l], offsets[l+1]) of shared next[] and
// keys[] arrays and starts at heads[l].  All lists are ranked at once as a
// forest: level 0 has one head chain per list (chain l) and one chain per
// node index multiple of 16 (chain H + j/16); level k >= 1 has one head chain
// per list (elements 0..H-1) and one chain per element x >= H with
// (x - H) mod 8 = 7.  The element ids of the non-head chains shrink by 8 per
// level, so after about log8(nodes / 16) levels only the H head chains are
// left, each covering its whole list, and the list offsets seed the offsets
// down the levels.  The lists then sit in list order at their own slab
// positions; stable passes on the key patterns followed by stable passes on
// the list id give every list its sorted run in its slab, and the relink
// closes each run with NIL.  Every step is one launch over all lists.
#include "pbit_device.h"
#include "pbit_launch.h"

namespace pbit {

struct ForestArgs {
    const uint32_t* heads;
    const uint64_t* offsets;
    uint32_t H;
    uint32_t n;
    LidMap lm;
    const uint32_t* head_bits;
    // gather form: per-list arrays with list-local indices (null otherwise)
    const uint64_t* next_in_ptrs;
    const uint64_t* next_out_ptrs;
    const uint64_t* key_ptrs;
};

// Head of list l as a batch node index (gather form: the head is list-local).
__device__ __forceinline__ uint32_t head_of(const ForestArgs& F, uint32_t l, uint64_t lo)
{
    const uint32_t h = F.heads[l];
    if (!F.next_in_ptrs || h == kNil)
        return h;
    return (uint32_t)min<uint64_t>(lo + h, (uint64_t)kNil);
}

__device__ __forceinline__ bool is_head(const ForestArgs& F, uint32_t node)
{
    return (F.head_bits[node >> 5] >> (node & 31)) & 1u;
}

// Per list: check its slab and head, mark the head, add its hash to the
// in-degree sums, count the NIL it must end with, fill the node->list table
// and count its nodes into the list-id histograms.
__global__ __launch_bounds__(256) void k_fprep(ForestArgs F, uint32_t* __restrict__ table,
                                               uint32_t* __restrict__ head_bits,
                                               uint32_t* __restrict__ hist, uint32_t key_passes,
                                               uint32_t lid_passes, uint32_t rb, Header* hdr)
{
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= F.H)
        return;
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    const uint32_t head = hi >= lo ? head_of(F, l, lo) : kNil;
    bool ok = hi >= lo && hi <= F.n && (l != 0 || lo == 0) && (l + 1 != F.H || hi == F.n);
    if (ok && hi == lo)
        ok = head == kNil;
    else if (ok)
        ok = head >= lo && head < hi;
    if (!ok) {
        set_error(&hdr->status, PBIT_EINVAL);
        return;
    }
    const uint32_t radix = 1u << rb;
    for (uint32_t q = 0; q < lid_passes; q++)
        if (hi > lo)
            atomicAdd(&hist[(key_passes + q) * radix + ((l >> (q * rb)) & (radix - 1u))],
                      (uint32_t)(hi - lo));
    if (hi == lo)
        return;
    atomicOr(&head_bits[head >> 5], 1u << (head & 31));
    atomicAdd((unsigned long long*)&hdr->hsum[0], (unsigned long long)mix64(head + 1ull, kHashK1));
    atomicAdd((unsigned long long*)&hdr->hsum[1], (unsigned long long)mix64(head + 1ull, kHashK2));
    atomicAdd(&hdr->expect_nil, 1u);
    const uint64_t B = 1ull << F.lm.log_block;
    for (uint64_t b = (lo + B - 1) / B; b < (hi + B - 1) / B; b++)
        table[b] = l;
}

__device__ __forceinline__ bool forest_shape_ok(const Header* hdr)
{
    return hdr->status == 0 && hdr->nil_count == hdr->expect_nil && hdr->hsum[0] == 0 &&
           hdr->hsum[1] == 0;
}

// Level 0 over all lists (see k_walk0 of the single-list path); a step that
// leaves the chain's slab marks the batch malformed.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_fwalk0(const NodeRec<KeyT>* __restrict__ nodes,
                                                ForestArgs F, uint32_t n_static,
                                                uint2* __restrict__ chain_rec,
                                                Entry<KeyT>* __restrict__ ent,
                                                uint32_t* __restrict__ resume, uint32_t cap,
                                                uint32_t* __restrict__ long_list, Header* hdr)
{
    constexpr uint32_t C = SegLen<KeyT>::value;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    if (!forest_shape_ok(hdr)) {
        if (c == 0 && hdr->status == 0)
            set_error(&hdr->status, PBIT_EMALFORMED);
        return;
    }
    const uint32_t n = F.n;
    uint32_t start;
    uint64_t lo, hi;
    if (c < F.H) {
        lo = F.offsets[c];
        hi = F.offsets[c + 1];
        if (lo == hi) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        start = head_of(F, c, lo);
    } else {
        const uint64_t j = (uint64_t)(c - F.H) << kLog0;
        if (j >= n || is_head(F, (uint32_t)j)) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        start = (uint32_t)j;
        const uint32_t l = list_of(F.lm, start);
        lo = F.offsets[l];
        hi = F.offsets[l + 1];
    }
    const uint32_t lmask = (1u << kLog0) - 1u;
    uint32_t cur = start, len = 0, nx = kNil;
    bool stop = false, bad = false;
    // register blocks of C entries, each stored in one burst (see k_walk0)
    while (!stop && len < cap) {
        Entry<KeyT> e[C];
        uint32_t got = 0;
#pragma unroll
        for (uint32_t t = 0; t < C; t++) {
            if (!stop) {
                const NodeRec<KeyT> r = nodes[cur];
                e[t].key = r.key;
                e[t].idx = cur;
                if constexpr (sizeof(KeyT) == 8) e[t].pad = 0;
                got = t + 1;
                nx = r.next;
                if (nx == kNil || (nx & lmask) == 0 || len + got >= n) {
                    stop = true;
                } else if (nx < lo || nx >= hi) {
                    bad = stop = true;
                } else {
                    cur = nx;
                }
            }
        }
#pragma unroll
        for (uint32_t t = 0; t < C; t++)
            if (t < got)
                ent[ent_at(n_static, c, len + t)] = e[t];
        len += got;
    }
    const uint32_t rest_from = stop ? kNil : cur;
    while (!stop) {
        nx = nodes[cur].next;
        len++;
        if (nx == kNil || (nx & lmask) == 0 || len >= n)
            stop = true;
        else if (nx < lo || nx >= hi)
            bad = stop = true;
        else
            cur = nx;
    }
    if (nx != kNil && (nx < lo || nx >= hi))
        bad = true;
    if (bad) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        nx = kNil;
    }
    record_long_chain(c, len, cap, rest_from, resume, long_list, hdr);
    chain_rec[c] = make_uint2(nx == kNil ? kNil : F.H + (nx >> kLog0), len);
}

// Start element of chain c at a level >= 1 with m elements (kNil: none).
__device__ __forceinline__ uint32_t fchain_start(uint32_t c, uint32_t H, uint32_t m)
{
    if (c < H)
        return c;
    const uint64_t x = (uint64_t)H + 8ull * (c - H) + 7ull;
    return x < m ? (uint32_t)x : kNil;
}

__device__ __forceinline__ bool fsplitter(uint32_t x, uint32_t H)
{
    return x < H || ((x - H) & 7u) == 7u;
}

__global__ __launch_bounds__(256) void k_fwalk_up(const uint2* __restrict__ recs, uint32_t m,
                                                  uint32_t H, uint32_t n_static,
                                                  uint2* __restrict__ chain_rec, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    const uint32_t start = fchain_start(c, H, m);
    if (start == kNil || recs[start].y == 0) {
        chain_rec[c] = make_uint2(kNil, 0);
        return;
    }
    uint32_t cur = start, w = 0, nx = kNil;
    bool bad = false;
    for (uint32_t steps = 0;; steps++) {
        const uint2 r = recs[cur];
        if (r.y == 0 || steps >= m) {
            bad = true;
            break;
        }
        w += r.y;
        nx = r.x;
        if (nx == kNil)
            break;
        if (nx >= m || nx < H) {
            bad = true;
            break;
        }
        if (fsplitter(nx, H))
            break;
        cur = nx;
    }
    if (bad) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        nx = kNil;
    }
    chain_rec[c] = make_uint2(nx == kNil ? kNil : H + ((nx - H) >> 3), w);
}

// Top level: every list is one head chain that must end in NIL and hold all
// nodes of its slab; its offset is the slab start.
__global__ __launch_bounds__(256) void k_ftop(const uint2* __restrict__ recs, ForestArgs F,
                                              uint32_t* __restrict__ offn, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= F.H)
        return;
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    const uint2 r = recs[l];
    if (r.y != (uint32_t)(hi - lo) || (hi > lo && r.x != kNil)) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        return;
    }
    offn[l] = (uint32_t)lo;
}

__global__ __launch_bounds__(256) void k_fdown(const uint2* __restrict__ recs, uint32_t m,
                                               uint32_t H, uint32_t n_static,
                                               const uint2* __restrict__ chain_rec,
                                               const uint32_t* __restrict__ offn_chain,
                                               uint32_t* __restrict__ offn_elem, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    if (chain_rec[c].y == 0)
        return;
    uint32_t cur = fchain_start(c, H, m);
    if (cur == kNil)
        return;
    uint32_t off = offn_chain[c];
    for (uint32_t steps = 0; steps < m; steps++) {
        const uint2 r = recs[cur];
        offn_elem[cur] = off;
        off += r.y;
        const uint32_t nx = r.x;
        if (nx == kNil || nx >= m || fsplitter(nx, H))
            break;
        cur = nx;
    }
}

// next_out[order[j]] = order[j+1] inside each list's run, NIL at its end;
// the first node of each run is the list's new head.  In the gather form the
// result goes to each list's own array in list-local indices.
__global__ __launch_bounds__(256) void k_frelink(OrderSrc src, ForestArgs F,
                                                 uint32_t* __restrict__ next_out,
                                                 uint32_t* __restrict__ new_heads,
                                                 int32_t* __restrict__ d_status, const Header* hdr)
{
    const int32_t st = hdr->status;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0)
        *d_status = st;
    if (st != 0)
        return;
    if (j < F.H && F.offsets[j] == F.offsets[j + 1])
        new_heads[j] = kNil;
    if (j >= F.n)
        return;
    const uint32_t kind = hdr->final_kind;
    const uint32_t l = list_of(F.lm, j);
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    const uint32_t node = order_at(src, kind, j);
    const uint32_t succ = (j + 1 < hi) ? order_at(src, kind, j + 1) : kNil;
    if (node < lo || node >= hi)
        return;  // cannot happen for a sorted batch; keeps every write in bounds
    if (F.next_out_ptrs) {
        uint32_t* out = (uint32_t*)F.next_out_ptrs[l];
        out[node - lo] = succ == kNil ? kNil : (uint32_t)(succ - lo);
        if (j == lo)
            new_heads[l] = (uint32_t)(node - lo);
    } else {
        next_out[node] = succ;
        if (j == lo)
            new_heads[l] = node;
    }
}

__global__ void k_fempty(uint32_t* __restrict__ new_heads, uint32_t H, int32_t* d_status)
{
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < H)
        new_heads[l] = kNil;
    if (l == 0)
        *d_status = 0;
}

// ---------------------------------------------------------------- launch
template <typename KeyT>
static hipError_t launch_fwalk0(const Plan& P, const ForestArgs& F, char* ws, hipStream_t s)
{
    const LevelPlan& L = P.lv[0];
    hipLaunchKernelGGL((k_fwalk0<KeyT>), dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0,
                       s, (const NodeRec<KeyT>*)(ws + P.o_nodes), F, (uint32_t)L.n_static,
                       (uint2*)(ws + L.o_chain_rec), (Entry<KeyT>*)(ws + L.o_ent),
                       (uint32_t*)(ws + L.o_resume), L.cap, (uint32_t*)(ws + L.o_long),
                       (Header*)(ws + P.o_header));
    return hipGetLastError();
}

hipError_t enqueue_sort_lists(const Plan& P, const uint32_t* heads, const uint64_t* offsets,
                              const uint32_t* next_in, uint32_t* next_out, const void* keys,
                              const uint64_t* next_in_ptrs, const uint64_t* next_out_ptrs,
                              const uint64_t* key_ptrs, uint32_t* new_heads, int32_t* d_status,
                              char* ws, hipStream_t s, Prof* prof)
{
    hipError_t e;
    Header* hdr = (Header*)(ws + P.o_header);
    if (P.n == 0) {
        hipLaunchKernelGGL(k_fempty, dim3((P.num_lists + 255) / 256), dim3(256), 0, s, new_heads,
                           P.num_lists, d_status);
        return hipGetLastError();
    }
    ForestArgs F;
    F.heads = heads;
    F.offsets = offsets;
    F.H = P.num_lists;
    F.n = (uint32_t)P.n;
    F.lm.table = (const uint32_t*)(ws + P.o_table);
    F.lm.offsets = offsets;
    F.lm.num_lists = P.num_lists;
    F.lm.log_block = P.log_block;
    F.head_bits = (const uint32_t*)(ws + P.o_headbits);
    F.next_in_ptrs = next_in_ptrs;
    F.next_out_ptrs = next_out_ptrs;
    F.key_ptrs = key_ptrs;

    mark(prof, s, kStageZero);
    if ((e = launch_zero(P, ws, s)) != hipSuccess)
        return e;
    {
        const size_t words = (P.n + 31) / 32 + 1;
        const size_t want = (words + 255) / 256;
        hipLaunchKernelGGL(k_zero, dim3((uint32_t)(want < 4096 ? want : 4096)), dim3(256), 0, s,
                           (uint32_t*)(ws + P.o_headbits), words);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_fprep, dim3((P.num_lists + 255) / 256), dim3(256), 0, s, F,
                       (uint32_t*)(ws + P.o_table), (uint32_t*)(ws + P.o_headbits),
                       (uint32_t*)(ws + P.o_hist), P.key_passes, P.passes - P.key_passes, P.RB,
                       hdr);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    mark(prof, s, kStagePack);
    if (next_in_ptrs) {
        switch (P.key_bytes) {
        case 1: e = launch_pack_src<uint8_t>(P, GatherSrc<uint8_t>{F.lm, next_in_ptrs, key_ptrs}, ws, s); break;
        case 2: e = launch_pack_src<uint16_t>(P, GatherSrc<uint16_t>{F.lm, next_in_ptrs, key_ptrs}, ws, s); break;
        case 4: e = launch_pack_src<uint32_t>(P, GatherSrc<uint32_t>{F.lm, next_in_ptrs, key_ptrs}, ws, s); break;
        default: e = launch_pack_src<uint64_t>(P, GatherSrc<uint64_t>{F.lm, next_in_ptrs, key_ptrs}, ws, s); break;
        }
    } else {
        switch (P.key_bytes) {
        case 1: e = launch_pack<uint8_t>(P, next_in, keys, ws, s); break;
        case 2: e = launch_pack<uint16_t>(P, next_in, keys, ws, s); break;
        case 4: e = launch_pack<uint32_t>(P, next_in, keys, ws, s); break;
        default: e = launch_pack<uint64_t>(P, next_in, keys, ws, s); break;
        }
    }
    if (e != hipSuccess)
        return e;
    mark(prof, s, kStageWalk0);
    switch (P.key_bytes) {
    case 1: e = launch_fwalk0<uint8_t>(P, F, ws, s); break;
    case 2: e = launch_fwalk0<uint16_t>(P, F, ws, s); break;
    case 4: e = launch_fwalk0<uint32_t>(P, F, ws, s); break;
    default: e = launch_fwalk0<uint64_t>(P, F, ws, s); break;
    }
    if (e != hipSuccess)
        return e;
    for (int k = 1; k < P.levels; k++) {
        const LevelPlan& L = P.lv[k];
        const LevelPlan& Lp = P.lv[k - 1];
        mark(prof, s, kStageWalkUp);
        hipLaunchKernelGGL(k_fwalk_up, dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0, s,
                           (const uint2*)(ws + Lp.o_chain_rec), (uint32_t)L.m, P.num_lists,
                           (uint32_t)L.n_static, (uint2*)(ws + L.o_chain_rec), hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    {
        const LevelPlan& Lt = P.lv[P.levels - 1];
        mark(prof, s, kStageBase);
        hipLaunchKernelGGL(k_ftop, dim3((P.num_lists + 255) / 256), dim3(256), 0, s,
                           (const uint2*)(ws + Lt.o_chain_rec), F, (uint32_t*)(ws + Lt.o_offn),
                           hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    for (int k = P.levels - 1; k >= 1; k--) {
        const LevelPlan& L = P.lv[k];
        const LevelPlan& Lp = P.lv[k - 1];
        mark(prof, s, kStageDown);
        hipLaunchKernelGGL(k_fdown, dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0, s,
                           (const uint2*)(ws + Lp.o_chain_rec), (uint32_t)L.m, P.num_lists,
                           (uint32_t)L.n_static, (const uint2*)(ws + L.o_chain_rec),
                           (const uint32_t*)(ws + L.o_offn), (uint32_t*)(ws + Lp.o_offn), hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    switch (P.key_bytes) {
    case 1: e = launch_unchain<uint8_t>(P, ws, s, prof); break;
    case 2: e = launch_unchain<uint16_t>(P, ws, s, prof); break;
    case 4: e = launch_unchain<uint32_t>(P, ws, s, prof); break;
    default: e = launch_unchain<uint64_t>(P, ws, s, prof); break;
    }
    if (e != hipSuccess)
        return e;
    switch (P.key_bytes) {
    case 1: e = launch_passes<uint8_t, uint64_t>(P, ws, s, prof, F.lm); break;
    case 2: e = launch_passes<uint16_t, uint64_t>(P, ws, s, prof, F.lm); break;
    case 4: e = launch_passes<uint32_t, uint64_t>(P, ws, s, prof, F.lm); break;
    default: e = launch_passes<uint64_t, uint64_t>(P, ws, s, prof, F.lm); break;
    }
    if (e != hipSuccess)
        return e;
    {
        const uint64_t threads = P.n > P.num_lists ? P.n : P.num_lists;
        mark(prof, s, kStageRelink);
        const OrderSrc src = P.key_bytes == 8 ? order_src<uint64_t>(P, ws) : order_src<uint32_t>(P, ws);
        hipLaunchKernelGGL(k_frelink, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s,
                           src, F, next_out, new_heads, d_status, (const Header*)hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    mark(prof, s, kStageCount);
    return hipSuccess;
}

}  // namespace pbit
