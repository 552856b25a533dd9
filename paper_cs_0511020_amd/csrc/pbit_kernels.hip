// HIP kernels (gfx950) of the Pbit list sort.
//
// Path for one list of n nodes (the split/concatenate method of the paper's
// Sec. 3 and Sec. 5, reorganised for a wide machine):
//   pack       next[] and keys[] become one 8- or 16-byte record per node so a
//              walk step is one random access; the histograms of every K-bit
//              pattern are counted here (order-free).
//   walk0      sparse-ruler list ranking, level 0: every node whose index is a
//              multiple of 16 (and the head) starts a chain; one lane walks
//              each chain, gathering its (key, node) entries in register
//              blocks that it stores to the chain's slot in bursts.
//   walk_up    the same on the list of chains, recursively, until the list
//              fits one workgroup.
//   base       pointer jumping (Wyllie) in LDS over the last level.
//   down       offsets flow back down the levels.
//   unchain    chain contents are copied to list order as (key, node) pairs;
//              the rests of chains longer than their slot are walked again.
//   schedule   per-pass digit bases; passes whose pattern is constant are
//              skipped (the identity), the paper's "empty groups are omitted".
//   digit pass stable K-bit split per pattern, least significant first:
//              per-wave ranking (LDS lane masks or ballots), LDS tile
//              staging, decoupled look-back.  Least-significant-first stable
//              passes give the same order as the paper's
//              most-significant-first recursion (both are the stable sort by
//              the full key).
//   relink     next[order[j]] = order[j+1], the concatenation of Sec. 5.1.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbit.h"
#include "pbit_internal.h"

#include "pbit_device.h"
#include "pbit_launch.h"

namespace pbit {

uint32_t pass_tile(uint32_t key_bytes, uint32_t rb)
{
    (void)rb;  // one shape for every pattern width
    return key_bytes == 8 ? PassShape<uint64_t, 8>::block * PassShape<uint64_t, 8>::items
                          : PassShape<uint32_t, 8>::block * PassShape<uint32_t, 8>::items;
}

// A single list passes the in-degree check if exactly one next[] is NIL and
// the hash sums over next[] match all nodes but the head.
__device__ __forceinline__ bool list_shape_ok(const Header* hdr, uint32_t head)
{
    return hdr->status == 0 && hdr->nil_count == 1 &&
           hdr->hsum[0] + mix64(head + 1ull, kHashK1) == 0 &&
           hdr->hsum[1] + mix64(head + 1ull, kHashK2) == 0;
}

// ---------------------------------------------------------------- list ranking
// Sparse-ruler ranking (Helman & JaJa style).  At level k the elements
// 0..m-1 form a list from `head` (element 0 for k >= 1).  Chain 0 starts at
// the head, chain 1 + j/L at element j for every multiple j of L = 2^log_l
// other than the head; a chain runs up to the next chain start or NIL.  One
// thread walks one chain to its end: no atomics, and the hardware refills a
// wave slot as soon as a wave's chains are done.  A chain's record is
// {successor chain or NIL, weight}; the chains form the list of level k + 1.
//
// Level 0 stores the first `cap` (key, node) entries of its chain in the
// chain's slot (SegLen at a time, through registers) and records the node
// where a longer chain resumes; after ranking, unchain walks only those rests
// again.
// Levels >= 1 store nothing: their down pass walks the chain again.
//
// The walks assume every node has at most one predecessor.  Pack checks it
// with two 64-bit hash sums over next[] (probabilistic: a malformed list
// passes only if both sums collide), so every node is walked once and a bad
// list is almost always rejected before any walk starts.  Safety does not
// rest on that check: every walk is bounded by n steps, every index is
// checked against n before use, and the base verifies that the chain lengths
// add up to n from the head.

template <typename KeyT>
__global__ __launch_bounds__(256) void k_walk0(const NodeRec<KeyT>* __restrict__ nodes, uint32_t n,
                                               uint32_t head, uint32_t n_static,
                                               uint2* __restrict__ chain_rec,
                                               Entry<KeyT>* __restrict__ ent,
                                               uint32_t* __restrict__ resume, uint32_t cap,
                                               uint32_t* __restrict__ long_list, Header* hdr,
                                               uint32_t walk_blocks,
                                               const uint32_t* __restrict__ hist,
                                               uint32_t* __restrict__ dbase, uint32_t passes,
                                               uint32_t radix, uint32_t hi_from)
{
    constexpr uint32_t C = SegLen<KeyT>::value;
    if (blockIdx.x == walk_blocks) {
        // one extra block: the pass schedule needs only pack's histograms, so
        // it runs beside the walk instead of as a launch of its own
        schedule_body(hist, dbase, passes, n, radix, hdr, hi_from);
        return;
    }
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    if (!list_shape_ok(hdr, head)) {
        if (c == 0 && hdr->status == 0)
            set_error(&hdr->status, PBIT_EMALFORMED);
        return;
    }
    uint32_t start = head;
    if (c != 0) {
        const uint64_t s = (uint64_t)(c - 1) << kLog0;
        if (s >= n || (uint32_t)s == head) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        start = (uint32_t)s;
    }
    const uint32_t lmask = (1u << kLog0) - 1u;
    uint32_t cur = start, len = 0, nx = kNil;
    bool stop = false;
    // The slot fills C entries at a time: a block of steps keeps its entries
    // in registers and stores them in one burst afterwards.  (A store issued
    // between two steps would be waited for by the next step's load: loads
    // and stores share one completion counter.)  cap is a multiple of C.
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
                if (nx == kNil || nx >= n || (nx & lmask) == 0 || nx == head || len + got >= n)
                    stop = true;
                else
                    cur = nx;
            }
        }
#pragma unroll
        for (uint32_t t = 0; t < C; t++)
            if (t < got)
                ent[ent_at(n_static, c, len + t)] = e[t];
        len += got;
    }
    // beyond the slot the walk only counts; unchain walks this rest again
    const uint32_t rest_from = stop ? kNil : cur;
    while (!stop) {
        nx = nodes[cur].next;
        len++;
        if (nx == kNil || nx >= n || (nx & lmask) == 0 || nx == head || len >= n)
            stop = true;
        else
            cur = nx;
    }
    if (nx != kNil && nx >= n) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        nx = kNil;
    }
    record_long_chain(c, len, cap, rest_from, resume, long_list, hdr);
    const uint32_t succ = (nx == kNil) ? kNil : (nx == head ? 0u : 1u + (nx >> kLog0));
    chain_rec[c] = make_uint2(succ, len);
}

// Level >= 1: chains over the records {successor, weight} of level k.
__global__ __launch_bounds__(256) void k_walk_up(const uint2* __restrict__ recs, uint32_t m,
                                                 uint32_t log_l, uint32_t n_static,
                                                 uint2* __restrict__ chain_rec, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    uint32_t start = 0;
    if (c != 0) {
        const uint64_t s = (uint64_t)(c - 1) << log_l;
        if (s >= m || s == 0) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        start = (uint32_t)s;
    }
    // A start element with no nodes is an empty chain of the level below (the
    // chain slot of a start node that is the head): this chain is empty too.
    // Only the head chain must not be empty.
    if (recs[start].y == 0) {
        if (c == 0)
            set_error(&hdr->status, PBIT_EMALFORMED);
        chain_rec[c] = make_uint2(kNil, 0);
        return;
    }
    const uint32_t lmask = (1u << log_l) - 1u;
    uint32_t cur = start, w = 0, steps = 0, nx;
    for (;;) {
        const uint2 r = recs[cur];
        if (r.y == 0) {  // an empty chain reached from a list: malformed
            set_error(&hdr->status, PBIT_EMALFORMED);
            nx = kNil;
            break;
        }
        w += r.y;
        nx = r.x;
        if (nx == kNil || nx >= m || (nx & lmask) == 0 || ++steps >= m)
            break;
        cur = nx;
    }
    if (nx != kNil && (nx >= m || steps >= m)) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        nx = kNil;
    }
    chain_rec[c] = make_uint2(nx == kNil ? kNil : (nx == 0 ? 0u : 1u + (nx >> log_l)), w);
}

// ---------------------------------------------------------------- base
// Pointer jumping (Wyllie) in LDS: suffix weights from every element to the
// end of the list, then offset = total - suffix.  The list must end in NIL
// from element 0 and cover exactly n nodes.  Each element is one 8-byte LDS
// word (pointer, weight); a thread keeps its own elements in registers, so a
// round is one dependent read and one write per element.
constexpr int kBaseThreads = 1024;
constexpr int kBasePer = kBaseMax / kBaseThreads;

__global__ __launch_bounds__(kBaseThreads) void k_base(const uint2* __restrict__ rec, uint32_t m,
                                                       uint32_t n_total,
                                                       uint32_t* __restrict__ offn, Header* hdr)
{
    __shared__ uint2 s_pv[kBaseMax];  // (pointer, suffix weight so far)
    __shared__ int s_bad;
    if (hdr->status != 0)
        return;
    m = min(m, kBaseMax);
    const int tid = threadIdx.x;
    if (tid == 0)
        s_bad = 0;
    uint2 own[kBasePer];
#pragma unroll
    for (int j = 0; j < kBasePer; j++) {
        const uint32_t i = tid + j * kBaseThreads;
        uint32_t p = kNil, v = 0;
        if (i < m) {
            const uint2 r = rec[i];
            if (r.y != 0) {
                p = (r.x != kNil && r.x >= m) ? kNil : r.x;  // caught below: total != n
                v = r.y;
            }
        }
        own[j] = make_uint2(p, v);
        s_pv[i] = own[j];
    }
    __syncthreads();
    int rounds = 1;
    while ((1u << (rounds - 1)) < m)
        rounds++;
    for (int r = 0; r < rounds; r++) {
#pragma unroll
        for (int j = 0; j < kBasePer; j++) {
            if (own[j].x != kNil) {
                const uint2 q = s_pv[own[j].x];
                own[j] = make_uint2(q.x, own[j].y + q.y);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kBasePer; j++)
            s_pv[tid + j * kBaseThreads] = own[j];
        __syncthreads();
    }
    const uint2 head = s_pv[0];
    const uint32_t total = head.y;
    if (tid == 0 && (m == 0 || head.x != kNil || total != n_total)) {
        s_bad = 1;
        set_error(&hdr->status, PBIT_EMALFORMED);
    }
    __syncthreads();
    if (s_bad)
        return;
#pragma unroll
    for (int j = 0; j < kBasePer; j++) {
        const uint32_t i = tid + j * kBaseThreads;
        if (i < m)
            offn[i] = total - own[j].y;
    }
}

// ---------------------------------------------------------------- down
// Level k >= 1: walk each chain again, giving each element its offset
// (chain offset plus the weights before it).
__global__ __launch_bounds__(256) void k_down(const uint2* __restrict__ recs, uint32_t m,
                                              uint32_t log_l, uint32_t n_static,
                                              const uint2* __restrict__ chain_rec,
                                              const uint32_t* __restrict__ offn_chain,
                                              uint32_t* __restrict__ offn_elem, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    const uint2 cr = chain_rec[c];
    if (cr.y == 0)
        return;
    const uint32_t start = c == 0 ? 0u : (c - 1) << log_l;
    const uint32_t lmask = (1u << log_l) - 1u;
    uint32_t cur = start, off = offn_chain[c];
    for (uint32_t steps = 0; steps < m; steps++) {
        const uint2 r = recs[cur];
        offn_elem[cur] = off;
        off += r.y;
        const uint32_t nx = r.x;
        if (nx == kNil || nx >= m || (nx & lmask) == 0)
            break;
        cur = nx;
    }
}

// ---------------------------------------------------------------- relink
// next[order[j]] = order[j+1]; the last node gets NIL; result = {head, status}.
// next_out: node i's new link goes to the uint32 at out_base + i * out_stride
// (a plain array: stride 4; records: the record stride).
__global__ __launch_bounds__(256) void k_relink(OrderSrc src, uint32_t n,
                                                char* __restrict__ out_base, uint64_t out_stride,
                                                uint32_t* __restrict__ result, const Header* hdr)
{
    const int32_t st = hdr->status;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (st != 0) {
        if (j == 0) {
            result[0] = kNil;
            result[1] = (uint32_t)st;
        }
        return;
    }
    const uint32_t kind = hdr->final_kind;
    if (j < n) {
        const uint32_t node = order_at(src, kind, j);
        const uint32_t succ = (j + 1 < n) ? order_at(src, kind, j + 1) : kNil;
        if (node < n)
            *(uint32_t*)(out_base + (uint64_t)node * out_stride) = succ;
        if (j == 0) {
            result[0] = node;
            result[1] = 0;
        }
    }
}

// Relink by node ranges.  The direct scatter writes each link at a random
// node, one 4-byte write per node anywhere in next[].  Instead:
//   1. k_relink_bucket: each tile of kRelinkTile list positions forms its
//      (node, successor) pairs and groups them in LDS by the node's range
//      (node >> r), written back over the tile's own span of a pairs buffer,
//      with the first slot of every range in the tile ([range][tile]);
//   2. k_relink_ranges: one workgroup per range of 2^r nodes gathers that
//      range's pairs from every tile into LDS, then writes the range's links
//      out in node order (coalesced).
// The result is the same array; the writes to next[] become sequential.
constexpr int kRelinkThreads = 1024;
constexpr int kRelinkItems = (int)kRelinkTile / kRelinkThreads;

__global__ __launch_bounds__(kRelinkThreads) void k_relink_bucket(
    OrderSrc src, uint32_t n, uint32_t r, uint32_t nranges, uint32_t ntiles,
    uint2* __restrict__ pairsA, uint2* __restrict__ pairsB, uint32_t* __restrict__ rstart,
    uint32_t* __restrict__ result, const Header* hdr)
{
    __shared__ uint32_t s_cnt[kRelinkRangesMax + 1];
    __shared__ uint32_t s_wsum[kRelinkThreads / 64];
    __shared__ __attribute__((aligned(16))) uint2 s_pairs[kRelinkTile];
    const int32_t st = hdr->status;
    const uint32_t kind = hdr->final_kind;
    const uint32_t tid = threadIdx.x, t = blockIdx.x;
    const uint64_t base = (uint64_t)t * kRelinkTile;
    const uint32_t cnt = (uint32_t)min<uint64_t>(kRelinkTile, (uint64_t)n - base);
    // the tile's order is loaded together with the status, from the index
    // buffer the last pass writes; it is loaded again from where it is when
    // no pass ran
    uint32_t node[kRelinkItems], succ[kRelinkItems], slot[kRelinkItems];
#pragma unroll
    for (int i = 0; i < kRelinkItems; i++) {
        const uint32_t k = (uint32_t)i * kRelinkThreads + tid;
        const uint64_t j = base + k;
        node[i] = k < cnt ? src.idxA[j] : kNil;
        succ[i] = k < cnt && j + 1 < n ? src.idxA[j + 1] : kNil;
    }
    if (st != 0) {
        if (t == 0 && tid == 0) {
            result[0] = kNil;
            result[1] = (uint32_t)st;
        }
        return;
    }
    if (kind != kBufIdxA) {
#pragma unroll
        for (int i = 0; i < kRelinkItems; i++) {
            const uint32_t k = (uint32_t)i * kRelinkThreads + tid;
            const uint64_t j = base + k;
            node[i] = k < cnt ? order_at(src, kind, j) : kNil;
            succ[i] = k < cnt && j + 1 < n ? order_at(src, kind, j + 1) : kNil;
        }
    }
    // the pairs go to a buffer the order is not read from
    uint2* pairs = kind == kBufPairsA ? pairsB : pairsA;
    for (uint32_t i = tid; i <= kRelinkRangesMax; i += kRelinkThreads)
        s_cnt[i] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRelinkItems; i++) {
        slot[i] = 0;
        if (node[i] < n)
            slot[i] = atomicAdd(&s_cnt[node[i] >> r], 1u);  // any order inside a range
        else
            node[i] = kNil;
    }
    __syncthreads();
    // exclusive scan of the range counts (one entry per thread)
    const uint32_t lane = tid % 64, wave = tid / 64;
    const uint32_t v = tid < nranges ? s_cnt[tid] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t up = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += up;
    }
    if (lane == 63)
        s_wsum[wave] = incl;
    __syncthreads();
    uint32_t wbase = 0;
    for (uint32_t w = 0; w < wave; w++)
        wbase += s_wsum[w];
    __syncthreads();
    if (tid < nranges)
        s_cnt[tid] = wbase + incl - v;
    if (tid == 0)
        s_cnt[nranges] = cnt;
    __syncthreads();
    for (uint32_t b = tid; b <= nranges; b += kRelinkThreads)
        rstart[(size_t)b * ntiles + t] = s_cnt[b];
#pragma unroll
    for (int i = 0; i < kRelinkItems; i++)
        if (node[i] != kNil)
            s_pairs[s_cnt[node[i] >> r] + slot[i]] = make_uint2(node[i], succ[i]);
    __syncthreads();
    for (uint32_t k = tid; k < cnt; k += kRelinkThreads)
        pairs[base + k] = s_pairs[k];
    if (t == 0 && tid == 0) {
        result[0] = order_at(src, kind, 0);
        result[1] = 0;
    }
}

// One workgroup per range of R nodes: every tile's pairs of this range (a
// segment of about kRelinkTile / ranges pairs per tile, read kRelinkBlock
// pairs at a time, one or two tiles per thread) land in LDS at their node;
// then the range's links are written in node order.
constexpr uint32_t kRelinkBlock = 16;
template <int R>
__global__ __launch_bounds__(kRelinkThreads) void k_relink_ranges(
    const uint2* __restrict__ pairsA, const uint2* __restrict__ pairsB,
    const uint32_t* __restrict__ rstart, uint32_t n, uint32_t ntiles,
    char* __restrict__ out_base, uint64_t out_stride, const Header* hdr)
{
    __shared__ uint32_t s_next[R];
    const uint32_t b = blockIdx.x, tid = threadIdx.x;
    const uint32_t* s0 = rstart + (size_t)b * ntiles;
    const uint32_t* s1 = rstart + (size_t)(b + 1) * ntiles;
    // the first tile's segment bounds are loaded together with the status
    const uint32_t a0 = tid < ntiles ? s0[tid] : 0u;
    const uint32_t e0 = tid < ntiles ? s1[tid] : 0u;
    if (hdr->status != 0)
        return;
    const uint2* pairs = hdr->final_kind == kBufPairsA ? pairsB : pairsA;
    const uint64_t lo = (uint64_t)b * R;
    const uint32_t len = (uint32_t)min<uint64_t>(R, (uint64_t)n - lo);
    for (uint32_t t = tid; t < ntiles; t += kRelinkThreads) {
        const uint32_t a = t == tid ? a0 : s0[t];
        const uint32_t e = min(t == tid ? e0 : s1[t], kRelinkTile);
        const uint2* p = pairs + (uint64_t)t * kRelinkTile;
        for (uint32_t k0 = a; k0 < e; k0 += kRelinkBlock) {
            uint2 q[kRelinkBlock];
#pragma unroll
            for (uint32_t u = 0; u < kRelinkBlock; u++)
                if (k0 + u < e)
                    q[u] = p[k0 + u];
#pragma unroll
            for (uint32_t u = 0; u < kRelinkBlock; u++) {
                if (k0 + u < e) {
                    const uint32_t loc = q[u].x - (uint32_t)lo;
                    if (loc < len)
                        s_next[loc] = q[u].y;
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < len; i += kRelinkThreads)
        *(uint32_t*)(out_base + (lo + i) * out_stride) = s_next[i];
}

__global__ void k_empty_result(uint32_t* result)
{
    result[0] = kNil;
    result[1] = 0;
}

// ---------------------------------------------------------------- launch helpers
template <typename KeyT>
static hipError_t launch_walk0(const Plan& P, uint32_t head, char* ws, hipStream_t s)
{
    const LevelPlan& L = P.lv[0];
    const uint32_t walk_blocks = (uint32_t)((L.n_static + 255) / 256);
    hipLaunchKernelGGL((k_walk0<KeyT>), dim3(walk_blocks + 1), dim3(256), 0, s,
                       (const NodeRec<KeyT>*)(ws + P.o_nodes), (uint32_t)P.n, head,
                       (uint32_t)L.n_static, (uint2*)(ws + L.o_chain_rec),
                       (Entry<KeyT>*)(ws + L.o_ent), (uint32_t*)(ws + L.o_resume), L.cap,
                       (uint32_t*)(ws + L.o_long), (Header*)(ws + P.o_header), walk_blocks,
                       (const uint32_t*)(ws + P.o_hist), (uint32_t*)(ws + P.o_dbase), P.passes,
                       P.radix, P.hi_from);
    return hipGetLastError();
}

// Everything after pack: ranking, list order, passes, relink.
static hipError_t enqueue_after_pack(const Plan& P, uint32_t head, char* out_base,
                                     uint64_t out_stride, uint32_t* d_result, char* ws,
                                     hipStream_t s, Prof* prof);

// ---------------------------------------------------------------- short list
// A list of at most CUT nodes (and at most the tuned cutoff): the whole sort
// by one workgroup in LDS (small_sort), one launch instead of the device-wide
// path.  Every link is read before any is written, so next_out may be
// next_in.  A malformed list leaves next_out untouched; the result is
// {new head, PBIT_OK} or {NIL, PBIT_EMALFORMED}, as from the relink.
template <typename KeyT, int RB, int CUT>
__global__ __launch_bounds__(kSmallThreads) void k_small_list(uint32_t head,
                                                              const uint32_t* next_in,
                                                              uint32_t* next_out, const KeyT* keys,
                                                              uint32_t n, KeyT float_sel,
                                                              KeyT xor_mask, uint32_t passes,
                                                              uint32_t* __restrict__ result)
{
    const uint32_t* links;
    uint32_t new_head;
    if (!small_sort<KeyT, RB, CUT>(next_in, keys, n, 0u, head, float_sel, xor_mask, passes, links,
                                   new_head)) {
        if (threadIdx.x == 0) {
            result[0] = kNil;
            result[1] = (uint32_t)PBIT_EMALFORMED;
        }
        return;
    }
    for (uint32_t i = threadIdx.x; i < n; i += kSmallThreads)
        next_out[i] = links[i];
    if (threadIdx.x == 0) {
        result[0] = new_head;
        result[1] = 0;
    }
}

constexpr uint32_t kSmallListMax = 4096;

template <typename KeyT, int RB>
static hipError_t launch_small_rb(const Plan& P, uint32_t head, const uint32_t* next_in,
                                  uint32_t* next_out, const void* keys, uint32_t* d_result,
                                  hipStream_t s)
{
    const KeyT float_sel = key_float_sel<KeyT>(P.flags), mask = key_xor_mask<KeyT>(P.flags);
    if (P.n <= 1024)
        hipLaunchKernelGGL((k_small_list<KeyT, RB, 1024>), dim3(1), dim3(kSmallThreads), 0, s,
                           head, next_in, next_out, (const KeyT*)keys, (uint32_t)P.n, float_sel,
                           mask, P.passes, d_result);
    else
        hipLaunchKernelGGL((k_small_list<KeyT, RB, kSmallListMax>), dim3(1), dim3(kSmallThreads),
                           0, s, head, next_in, next_out, (const KeyT*)keys, (uint32_t)P.n,
                           float_sel, mask, P.passes, d_result);
    return hipGetLastError();
}

template <typename KeyT>
static hipError_t launch_small(const Plan& P, uint32_t head, const uint32_t* next_in,
                               uint32_t* next_out, const void* keys, uint32_t* d_result,
                               hipStream_t s)
{
    switch (P.RB) {
    case 1: return launch_small_rb<KeyT, 1>(P, head, next_in, next_out, keys, d_result, s);
    case 2: return launch_small_rb<KeyT, 2>(P, head, next_in, next_out, keys, d_result, s);
    case 4: return launch_small_rb<KeyT, 4>(P, head, next_in, next_out, keys, d_result, s);
    default: return launch_small_rb<KeyT, 8>(P, head, next_in, next_out, keys, d_result, s);
    }
}

// The whole path queued on one stream.
hipError_t enqueue_sort(const Plan& P, uint32_t head, const uint32_t* next_in, uint32_t* next_out,
                        const void* keys, uint32_t* d_result, char* ws, hipStream_t s, Prof* prof)
{
    hipError_t e;
    if (P.n <= P.cutoff && P.n <= kSmallListMax) {
        mark(prof, s, kStageSmall);
        switch (P.key_bytes) {
        case 1: e = launch_small<uint8_t>(P, head, next_in, next_out, keys, d_result, s); break;
        case 2: e = launch_small<uint16_t>(P, head, next_in, next_out, keys, d_result, s); break;
        case 4: e = launch_small<uint32_t>(P, head, next_in, next_out, keys, d_result, s); break;
        default: e = launch_small<uint64_t>(P, head, next_in, next_out, keys, d_result, s); break;
        }
        if (e == hipSuccess)
            mark(prof, s, kStageCount);
        return e;
    }
    mark(prof, s, kStageZero);
    if ((e = launch_zero(P, ws, s)) != hipSuccess)
        return e;
    mark(prof, s, kStagePack);
    switch (P.key_bytes) {
    case 1: e = launch_pack<uint8_t>(P, next_in, keys, ws, s); break;
    case 2: e = launch_pack<uint16_t>(P, next_in, keys, ws, s); break;
    case 4: e = launch_pack<uint32_t>(P, next_in, keys, ws, s); break;
    default: e = launch_pack<uint64_t>(P, next_in, keys, ws, s); break;
    }
    if (e != hipSuccess)
        return e;
    return enqueue_after_pack(P, head, (char*)next_out, 4, d_result, ws, s, prof);
}

// The same for nodes stored as records; the links are rewritten in place.
hipError_t enqueue_sort_aos(const Plan& P, uint32_t head, char* base, uint64_t stride,
                            uint32_t next_off, uint32_t key_off, uint32_t* d_result, char* ws,
                            hipStream_t s, Prof* prof)
{
    hipError_t e;
    mark(prof, s, kStageZero);
    if ((e = launch_zero(P, ws, s)) != hipSuccess)
        return e;
    mark(prof, s, kStagePack);
    switch (P.key_bytes) {
    case 1: e = launch_pack_src<uint8_t>(P, AosSrc<uint8_t>{base, stride, next_off, key_off}, ws, s); break;
    case 2: e = launch_pack_src<uint16_t>(P, AosSrc<uint16_t>{base, stride, next_off, key_off}, ws, s); break;
    case 4: e = launch_pack_src<uint32_t>(P, AosSrc<uint32_t>{base, stride, next_off, key_off}, ws, s); break;
    default: e = launch_pack_src<uint64_t>(P, AosSrc<uint64_t>{base, stride, next_off, key_off}, ws, s); break;
    }
    if (e != hipSuccess)
        return e;
    return enqueue_after_pack(P, head, base + next_off, stride, d_result, ws, s, prof);
}

static hipError_t enqueue_after_pack(const Plan& P, uint32_t head, char* out_base,
                                     uint64_t out_stride, uint32_t* d_result, char* ws,
                                     hipStream_t s, Prof* prof)
{
    hipError_t e;
    mark(prof, s, kStageWalk0);
    switch (P.key_bytes) {
    case 1: e = launch_walk0<uint8_t>(P, head, ws, s); break;
    case 2: e = launch_walk0<uint16_t>(P, head, ws, s); break;
    case 4: e = launch_walk0<uint32_t>(P, head, ws, s); break;
    default: e = launch_walk0<uint64_t>(P, head, ws, s); break;
    }
    if (e != hipSuccess)
        return e;
    Header* hdr = (Header*)(ws + P.o_header);
    for (int k = 1; k < P.levels; k++) {
        const LevelPlan& L = P.lv[k];
        const LevelPlan& Lp = P.lv[k - 1];
        mark(prof, s, kStageWalkUp);
        hipLaunchKernelGGL(k_walk_up, dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0, s,
                           (const uint2*)(ws + Lp.o_chain_rec), (uint32_t)L.m, L.log_l,
                           (uint32_t)L.n_static, (uint2*)(ws + L.o_chain_rec), hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    {
        const LevelPlan& Lt = P.lv[P.levels - 1];
        mark(prof, s, kStageBase);
        hipLaunchKernelGGL(k_base, dim3(1), dim3(kBaseThreads), 0, s,
                           (const uint2*)(ws + Lt.o_chain_rec), (uint32_t)Lt.n_static,
                           (uint32_t)P.n, (uint32_t*)(ws + Lt.o_offn), hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    for (int k = P.levels - 1; k >= 1; k--) {
        const LevelPlan& L = P.lv[k];
        const LevelPlan& Lp = P.lv[k - 1];
        mark(prof, s, kStageDown);
        hipLaunchKernelGGL(k_down, dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0, s,
                           (const uint2*)(ws + Lp.o_chain_rec), (uint32_t)L.m, L.log_l,
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
    if (P.look64) {
        switch (P.key_bytes) {
        case 1: e = launch_passes<uint8_t, uint64_t, false>(P, ws, s, prof, true); break;
        case 2: e = launch_passes<uint16_t, uint64_t, false>(P, ws, s, prof, true); break;
        case 4: e = launch_passes<uint32_t, uint64_t, false>(P, ws, s, prof, true); break;
        default: e = launch_passes<uint64_t, uint64_t, false>(P, ws, s, prof, true); break;
        }
    } else {
        switch (P.key_bytes) {
        case 1: e = launch_passes<uint8_t, uint32_t, false>(P, ws, s, prof, true); break;
        case 2: e = launch_passes<uint16_t, uint32_t, false>(P, ws, s, prof, true); break;
        case 4: e = launch_passes<uint32_t, uint32_t, false>(P, ws, s, prof, true); break;
        default: e = launch_passes<uint64_t, uint32_t, false>(P, ws, s, prof, true); break;
        }
    }
    if (e != hipSuccess)
        return e;
    {
        uint32_t blocks = (uint32_t)((P.n + 255) / 256);
        mark(prof, s, kStageRelink);
        const OrderSrc src = P.key_bytes == 8 ? order_src<uint64_t>(P, ws) : order_src<uint32_t>(P, ws);
        if (P.relink_r != 0) {
            hipLaunchKernelGGL(k_relink_bucket, dim3(P.relink_tiles), dim3(kRelinkThreads), 0, s,
                               src, (uint32_t)P.n, P.relink_r, P.relink_ranges, P.relink_tiles,
                               (uint2*)(ws + P.o_pairsA), (uint2*)(ws + P.o_pairsB),
                               (uint32_t*)(ws + P.o_rstart), d_result, (const Header*)hdr);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
            if (P.relink_r == 14)
                hipLaunchKernelGGL((k_relink_ranges<1 << 14>), dim3(P.relink_ranges),
                                   dim3(kRelinkThreads), 0, s, (const uint2*)(ws + P.o_pairsA),
                                   (const uint2*)(ws + P.o_pairsB),
                                   (const uint32_t*)(ws + P.o_rstart), (uint32_t)P.n,
                                   P.relink_tiles, out_base, out_stride, (const Header*)hdr);
            else
                hipLaunchKernelGGL((k_relink_ranges<1 << 15>), dim3(P.relink_ranges),
                                   dim3(kRelinkThreads), 0, s, (const uint2*)(ws + P.o_pairsA),
                                   (const uint2*)(ws + P.o_pairsB),
                                   (const uint32_t*)(ws + P.o_rstart), (uint32_t)P.n,
                                   P.relink_tiles, out_base, out_stride, (const Header*)hdr);
        } else {
            hipLaunchKernelGGL(k_relink, dim3(blocks), dim3(256), 0, s, src, (uint32_t)P.n,
                               out_base, out_stride, d_result, (const Header*)hdr);
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    mark(prof, s, kStageCount);
    return hipSuccess;
}

hipError_t enqueue_empty(uint32_t* d_result, hipStream_t s)
{
    hipLaunchKernelGGL(k_empty_result, dim3(1), dim3(1), 0, s, d_result);
    return hipGetLastError();
}

// Backward links of doubly-linked lists (Sec. 13).  Each node's backward link
// is fixed by its own forward link alone, so the walk from the head becomes one
// scatter: prev[next[i]] = i over every node, and NIL for every head.  next[]
// is read in index order (coalesced); the prev[] writes land in random lines.
// A non-zero status on entry (a sort that found a malformed list) leaves prev[]
// untouched; an index >= n is skipped and reported.
__global__ __launch_bounds__(256) void k_repair_prev(const uint32_t* __restrict__ heads,
                                                     uint32_t num_lists,
                                                     const uint32_t* __restrict__ next,
                                                     uint32_t* __restrict__ prev, uint32_t n,
                                                     int32_t* status)
{
    if (status && ld_agent(status) != 0)
        return;
    bool bad = false;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t i = tid; i < n; i += stride) {
        const uint32_t nx = next[i];
        if (nx == kNil)
            continue;
        if (nx < n)
            prev[nx] = i;
        else
            bad = true;
    }
    for (uint32_t l = tid; l < num_lists; l += stride) {
        const uint32_t h = heads[l];
        if (h == kNil)
            continue;
        if (h < n)
            prev[h] = kNil;
        else
            bad = true;
    }
    if (bad && status)
        set_error(status, PBIT_EMALFORMED);
}

hipError_t enqueue_repair_prev(const uint32_t* heads, uint32_t num_lists, const uint32_t* next,
                               uint32_t* prev, uint32_t n, int32_t* status, hipStream_t s)
{
    const uint64_t work = (uint64_t)(n > num_lists ? n : num_lists);
    const uint64_t want = (work + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 8192 ? (want ? want : 1) : 8192);
    hipLaunchKernelGGL(k_repair_prev, dim3(blocks), dim3(256), 0, s, heads, num_lists, next, prev,
                       n, status);
    return hipGetLastError();
}

}  // namespace pbit
