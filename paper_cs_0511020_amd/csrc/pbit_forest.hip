// Many independent lists sorted together (HIP, gfx950).
//
// List l owns the node slab [offsets[l], offsets[l+1]) of shared next[] and
// keys[] arrays (or, in the gather form, arrays of its own) and starts at
// heads[l].  Each list is split by K-bit patterns and concatenated as in the
// paper's Sec. 3 and Sec. 5, every list on its own; the batch only shares the
// launches.
//
// Two paths, chosen per list by its length against a cutoff (at least
// kMinSegLen nodes):
//  - a short list is sorted by one workgroup in LDS (k_fsmall): its links
//    and keys are read once, it is ranked by pointer jumping, sorted by
//    stable K-bit passes in LDS and its new links are written once;
//  - the long lists ("segments") are compacted, in list order, into one
//    position range each, list s at [coff[s], coff[s+1]).  They are ranked
//    together as a forest (level 0 has one head chain per list, chain l, and
//    one chain per node index multiple of 16, chain H + j/16; level k >= 1
//    has one head chain per list and one chain per element x >= H with
//    (x - H) mod 8 = 7, so after about log8(nodes / 16) levels only the head
//    chains remain, each covering its whole list), unchained into the
//    position array, and put through the stable digit passes with a base per
//    list and digit (k_digit_pass, SEG), which keeps every list inside its
//    own range: no pass on list ids is needed.  The per-list digit counts
//    come from pack; the bases from a scan over lists (k_lprep, k_lscan,
//    k_lfin).
// The relink closes every segment with NIL and a commit step copies the short
// lists' results out.  Every step is one launch over all lists, and no
// results are written before the whole batch is validated.
#include "pbit_device.h"
#include "pbit_launch.h"

namespace pbit {

struct ForestArgs {
    const uint32_t* heads;
    const uint64_t* offsets;
    uint32_t H;
    uint32_t n;
    uint32_t cutoff;           // lists longer than this are segments
    LidMap lm;                 // node -> list
    const uint32_t* head_bits;
    const uint32_t* lrank;     // lrank[l] = segments among lists before l (H + 1 entries)
    const uint32_t* segl;      // segment -> list
    const uint32_t* coff;      // segment -> first position (n_segs + 1 entries)
    // gather form: per-list arrays with list-local indices (null otherwise)
    const uint64_t* next_in_ptrs;
    const uint64_t* next_out_ptrs;
    const uint64_t* key_ptrs;
};

__device__ __forceinline__ bool is_seg(const ForestArgs& F, uint32_t l)
{
    return F.lrank[l + 1] != F.lrank[l];
}

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

// Exclusive scan of one value per thread over a block of 1024 threads.
__device__ __forceinline__ uint32_t block_excl_scan_1024(uint32_t v, uint32_t* s_tmp,
                                                         uint32_t& total)
{
    const uint32_t lane = __lane_id(), wave = threadIdx.x / 64;
    uint32_t incl = v;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t up = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += up;
    }
    if (lane == 63)
        s_tmp[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < 16; w++) {
            const uint32_t x = s_tmp[w];
            s_tmp[w] = run;
            run += x;
        }
        s_tmp[16] = run;
    }
    __syncthreads();
    const uint32_t r = s_tmp[wave] + incl - v;
    total = s_tmp[16];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- plan
// One block of 1024 threads over all lists: check every slab and head (a
// bad one makes the batch PBIT_EINVAL); number the segments (lists longer
// than the cutoff) in list order with their position ranges; mark and hash
// their heads and count the NILs they must end with (the in-degree check of
// pack covers segment nodes only: short lists are checked in LDS).
__global__ __launch_bounds__(1024) void k_fplan(ForestArgs F, uint32_t* __restrict__ lrank,
                                                uint32_t* __restrict__ segl,
                                                uint32_t* __restrict__ coff,
                                                uint32_t* __restrict__ head_bits, Header* hdr)
{
    __shared__ uint32_t s_tmp[17];
    const uint32_t T = blockDim.x;
    const uint32_t per = (F.H + T - 1) / T;
    const uint32_t l0 = min(threadIdx.x * per, F.H), l1 = min(l0 + per, F.H);
    uint32_t segs = 0, nodes = 0;
    bool bad = false;
    for (uint32_t l = l0; l < l1; l++) {
        const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
        bool ok = hi >= lo && hi <= F.n && (l != 0 || lo == 0) && (l + 1 != F.H || hi == F.n);
        const uint32_t head = ok ? head_of(F, l, lo) : kNil;
        if (ok && hi == lo)
            ok = head == kNil;
        else if (ok)
            ok = head >= lo && head < hi;
        bad |= !ok;
        if (ok && hi - lo > F.cutoff) {
            segs++;
            nodes += (uint32_t)(hi - lo);
        }
    }
    uint32_t tot_segs, tot_nodes;
    uint32_t seg = block_excl_scan_1024(segs, s_tmp, tot_segs);
    uint32_t pos = block_excl_scan_1024(nodes, s_tmp, tot_nodes);
    const int any_bad = __syncthreads_or(bad);
    if (any_bad) {
        if (threadIdx.x == 0)
            set_error(&hdr->status, PBIT_EINVAL);
        return;
    }
    uint64_t h1 = 0, h2 = 0;
    uint32_t nils = 0;
    for (uint32_t l = l0; l < l1; l++) {
        const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
        lrank[l] = seg;
        if (hi - lo > F.cutoff) {
            const uint32_t head = head_of(F, l, lo);
            segl[seg] = l;
            coff[seg] = pos;
            seg++;
            pos += (uint32_t)(hi - lo);
            atomicOr(&head_bits[head >> 5], 1u << (head & 31));
            h1 += mix64(head + 1ull, kHashK1);
            h2 += mix64(head + 1ull, kHashK2);
            nils++;
        }
    }
    if (threadIdx.x == 0) {
        lrank[F.H] = tot_segs;
        coff[tot_segs] = tot_nodes;
        hdr->n_segs = tot_segs;
        hdr->seg_nodes = tot_nodes;
    }
    if (nils) {
        atomicAdd((unsigned long long*)&hdr->hsum[0], (unsigned long long)h1);
        atomicAdd((unsigned long long*)&hdr->hsum[1], (unsigned long long)h2);
        atomicAdd(&hdr->expect_nil, nils);
    }
}

// One workgroup per list: the node -> list table over node indices and, for
// segments, the position -> segment table over their position ranges (both
// at 256-entry granularity: entry b names the list holding index b * 256).
__global__ __launch_bounds__(256) void k_ftables(ForestArgs F, uint32_t* __restrict__ table,
                                                 uint32_t* __restrict__ ctable, Header* hdr)
{
    const uint32_t l = blockIdx.x;
    if (l >= F.H || hdr->status != 0)
        return;
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    const uint64_t B = 1ull << F.lm.log_block;
    for (uint64_t b = (lo + B - 1) / B + threadIdx.x; b < (hi + B - 1) / B; b += blockDim.x)
        table[b] = l;
    if (is_seg(F, l)) {
        const uint32_t s = F.lrank[l];
        const uint64_t c0 = F.coff[s], c1 = c0 + (hi - lo);
        const uint64_t C = 1ull << kSegLog;
        for (uint64_t b = (c0 + C - 1) / C + threadIdx.x; b < (c1 + C - 1) / C; b += blockDim.x)
            ctable[b] = s;
    }
}

__device__ __forceinline__ bool forest_shape_ok(const Header* hdr)
{
    return hdr->status == 0 && hdr->nil_count == hdr->expect_nil && hdr->hsum[0] == 0 &&
           hdr->hsum[1] == 0;
}

// ---------------------------------------------------------------- pack
// Pack for the segments: records {next, transformed key} of segment nodes,
// the in-degree hash sums and NIL count over them, and every segment's digit
// counts for every pass.  A block takes a contiguous chunk of node indices;
// the first kPackSlots segments it meets count in LDS and flush once per
// (segment, pass, digit), any further ones (only when many lists just above
// the cutoff share a chunk) count with global atomics.  Nodes of short lists
// are left to k_fsmall.
template <typename KeyT, int RB, class Src>
__global__ __launch_bounds__(256) void k_fpack(Src src, ForestArgs F, uint32_t chunk,
                                               KeyT float_sel, KeyT xor_mask, uint32_t passes,
                                               uint32_t seg_max, NodeRec<KeyT>* __restrict__ nodes,
                                               uint32_t* __restrict__ lcnt, Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    extern __shared__ uint32_t s_hist[];  // kPackSlots * passes * RADIX
    if (__syncthreads_or(hdr->status != 0))
        return;
    const uint32_t per_slot = passes * RADIX;
    for (uint32_t i = threadIdx.x; i < kPackSlots * per_slot; i += blockDim.x)
        s_hist[i] = 0;
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = min<uint64_t>(c0 + chunk, (uint64_t)F.n);
    const uint32_t seg0 = c0 < F.n ? F.lrank[list_of(F.lm, (uint32_t)c0)] : 0u;
    __syncthreads();
    bool bad = false;
    uint64_t h1 = 0, h2 = 0;
    uint32_t nils = 0;
    // one segment node: key transform, hashes, NIL count, digit counts
    auto count = [&](uint64_t i, uint32_t nx, KeyT k, uint32_t s) -> KeyT {
        k = transform_key<KeyT>(k, float_sel, xor_mask);
        if (nx == kNil) {
            nils++;
        } else {
            h1 += mix64(nx + 1ull, kHashK1);
            h2 += mix64(nx + 1ull, kHashK2);
        }
        h1 -= mix64(i + 1ull, kHashK1);
        h2 -= mix64(i + 1ull, kHashK2);
        const uint32_t slot = s - seg0;
        for (uint32_t p = 0; p < passes; p++) {
            const uint32_t d = (uint32_t)(k >> (p * RB)) & (RADIX - 1u);
            if (slot < kPackSlots)
                atomicAdd(&s_hist[slot * per_slot + p * RADIX + d], 1u);
            else
                atomicAdd(&lcnt[((size_t)p * seg_max + s) * RADIX + d], 1u);
        }
        return k;
    };
    auto one = [&](uint64_t i, uint32_t s) {
        uint32_t nx;
        KeyT k;
        src.load(i, F.n, nx, k, bad);
        k = count(i, nx, k, s);
        NodeRec<KeyT> r;
        r.next = nx;
        r.key = k;
        if constexpr (sizeof(KeyT) == 8) r.pad = 0;
        nodes[i] = r;
    };
    // Each wave takes 256 consecutive nodes at a time, 4 per lane.  Usually
    // they all belong to one list: then the list is looked up once (and a
    // short list's nodes are skipped without a read), and 32-bit keys move
    // with 16-byte loads and 32-byte record stores.
    bool wide = false;
    if constexpr (Loads4<Src>::value)
        wide = (((uintptr_t)src.next | (uintptr_t)src.keys) & 15u) == 0;
    const uint32_t wave = threadIdx.x / 64, lane = __lane_id();
    for (uint64_t g0 = c0 + (uint64_t)wave * 256; g0 < c1; g0 += blockDim.x * 4ull) {
        const uint64_t g1 = min<uint64_t>(g0 + 256, c1);
        const uint32_t la = list_of(F.lm, (uint32_t)g0), lb = list_of(F.lm, (uint32_t)(g1 - 1));
        const uint64_t q0 = g0 + 4ull * lane;
        if (la == lb) {
            const uint32_t s = F.lrank[la];
            if (F.lrank[la + 1] == s)
                continue;  // a short list's nodes
            if constexpr (Loads4<Src>::value) {
                if (wide && q0 + 4 <= g1) {
                    const uint4 a = ((const uint4*)src.next)[q0 / 4];
                    const uint4 b = ((const uint4*)src.keys)[q0 / 4];
                    const uint32_t nx[4] = {a.x, a.y, a.z, a.w};
                    uint32_t k[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        bad |= (nx[j] != kNil) && (nx[j] >= F.n);
                        k[j] = count(q0 + j, nx[j], k[j], s);
                    }
                    uint4* out = (uint4*)(nodes + q0);
                    out[0] = make_uint4(nx[0], k[0], nx[1], k[1]);
                    out[1] = make_uint4(nx[2], k[2], nx[3], k[3]);
                    continue;
                }
            }
            for (uint64_t i = q0; i < min<uint64_t>(q0 + 4, g1); i++)
                one(i, s);
        } else {
            for (uint64_t i = q0; i < min<uint64_t>(q0 + 4, g1); i++) {
                const uint32_t l = list_of(F.lm, (uint32_t)i);
                const uint32_t s = F.lrank[l];
                if (F.lrank[l + 1] != s)
                    one(i, s);
            }
        }
    }
    if (bad)
        set_error(&hdr->status, PBIT_EMALFORMED);
    for (int off = 32; off > 0; off >>= 1) {
        h1 += (uint64_t)__shfl_xor((unsigned long long)h1, off, 64);
        h2 += (uint64_t)__shfl_xor((unsigned long long)h2, off, 64);
        nils += __shfl_xor(nils, off, 64);
    }
    __shared__ uint64_t s_h[2][4];
    __shared__ uint32_t s_nil[4];
    if (lane == 0) {
        s_h[0][wave] = h1;
        s_h[1][wave] = h2;
        s_nil[wave] = nils;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0;
        uint32_t z = 0;
        for (uint32_t w = 0; w < blockDim.x / 64; w++) {
            a += s_h[0][w];
            b += s_h[1][w];
            z += s_nil[w];
        }
        if (a | b) {
            atomicAdd((unsigned long long*)&hdr->hsum[0], (unsigned long long)a);
            atomicAdd((unsigned long long*)&hdr->hsum[1], (unsigned long long)b);
        }
        if (z)
            atomicAdd(&hdr->nil_count, z);
    }
    // only the slots of segments this chunk met
    const uint32_t used =
        c0 < c1 ? min(kPackSlots, F.lrank[list_of(F.lm, (uint32_t)(c1 - 1)) + 1] - seg0) : 0u;
    for (uint32_t i = threadIdx.x; i < used * per_slot; i += blockDim.x) {
        const uint32_t v = s_hist[i];
        if (v) {
            const uint32_t slot = i / per_slot, r = i % per_slot;
            const uint32_t p = r / RADIX, d = r % RADIX;
            atomicAdd(&lcnt[((size_t)p * seg_max + seg0 + slot) * RADIX + d], v);
        }
    }
}

// ---------------------------------------------------------------- short lists
// A list of at most CUT nodes is sorted by one workgroup in LDS (small_sort);
// its new links (list-local) go to snext in index order and its new head to
// shead; k_fcommit copies them to the caller's arrays once the whole batch is
// known to be valid.
template <typename KeyT, int RB, int CUT>
__global__ __launch_bounds__(kSmallThreads) void k_fsmall(ForestArgs F, const uint32_t* next_in,
                                                          const KeyT* keys, KeyT float_sel,
                                                          KeyT xor_mask, uint32_t passes,
                                                          uint32_t* __restrict__ snext,
                                                          uint32_t* __restrict__ shead,
                                                          Header* hdr)
{
    const uint32_t l = blockIdx.x;
    if (l >= F.H)
        return;
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    if (__syncthreads_or(ld_agent(&hdr->status) != 0))
        return;
    if (hi <= lo || hi - lo > CUT || hi - lo > F.cutoff)
        return;
    const uint32_t len = (uint32_t)(hi - lo);
    const uint32_t* nxt = F.next_in_ptrs ? (const uint32_t*)F.next_in_ptrs[l] : next_in + lo;
    const KeyT* kp = F.next_in_ptrs ? (const KeyT*)F.key_ptrs[l] : keys + lo;
    const uint32_t shift_in = F.next_in_ptrs ? 0u : (uint32_t)lo;  // global -> local
    // the head was checked against the slab before (k_fplan)
    const uint32_t h = head_of(F, l, lo) - (uint32_t)lo;
    const uint32_t* links;
    uint32_t new_head;
    if (!small_sort<KeyT, RB, CUT>(nxt, kp, len, shift_in, h, float_sel, xor_mask, passes, links,
                                   new_head)) {
        if (threadIdx.x == 0)
            set_error(&hdr->status, PBIT_EMALFORMED);
        return;
    }
    for (uint32_t i = threadIdx.x; i < len; i += kSmallThreads)
        snext[lo + i] = links[i];
    if (threadIdx.x == 0)
        shead[l] = new_head;
}

// ---------------------------------------------------------------- ranking
// Level 0 over the segments (see k_walk0 of the single-list path); a step
// that leaves the chain's slab marks the batch malformed.
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
        if (!is_seg(F, c)) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        lo = F.offsets[c];
        hi = F.offsets[c + 1];
        start = head_of(F, c, lo);
    } else {
        const uint64_t j = (uint64_t)(c - F.H) << kLog0;
        if (j >= n || is_head(F, (uint32_t)j)) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        start = (uint32_t)j;
        const uint32_t l = list_of(F.lm, start);
        if (!is_seg(F, l)) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
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

// Top level: every segment is one head chain that must end in NIL and hold
// all nodes of its slab; its offset is the start of its position range.
__global__ __launch_bounds__(256) void k_ftop(const uint2* __restrict__ recs, ForestArgs F,
                                              uint32_t* __restrict__ offn, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= F.H || !is_seg(F, l))
        return;
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    const uint2 r = recs[l];
    if (r.y != (uint32_t)(hi - lo) || r.x != kNil) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        return;
    }
    offn[l] = F.coff[F.lrank[l]];
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

// ---------------------------------------------------------------- per-list bases
// lbase[p][s][d] = coff[s] + (count of digit < d in segment s) - (count of
// digit d in segments before s), from the per-segment counts lcnt[p][s][d].
// k_lprep: blocks [0, row_blocks) give one wave per (pass, segment) row: the
// row's exclusive scan over digits plus coff[s], and whether the row has a
// single digit (the pass is the identity for that list).  The other blocks
// give one thread per (pass, group of kSegChunk segments, digit): the
// group's column sum.
template <int RB>
__global__ __launch_bounds__(256) void k_lprep(const uint32_t* __restrict__ lcnt,
                                               uint32_t* __restrict__ lbase,
                                               uint32_t* __restrict__ csum,
                                               const uint32_t* __restrict__ coff,
                                               uint32_t passes, uint32_t seg_max,
                                               uint32_t seg_chunks, uint32_t row_blocks,
                                               Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    if (hdr->status != 0)
        return;
    const uint32_t nseg = hdr->n_segs;
    if (blockIdx.x < row_blocks) {
        const uint32_t row = blockIdx.x * 4 + threadIdx.x / 64;
        const uint32_t p = row / seg_max, s = row % seg_max;
        if (p >= passes || s >= nseg)
            return;
        const uint32_t lane = __lane_id();
        const uint32_t len = coff[s + 1] - coff[s];
        constexpr uint32_t PER = (RADIX + 63) / 64;
        const uint32_t* rowp = lcnt + ((size_t)p * seg_max + s) * RADIX;
        uint32_t vals[PER], local = 0;
        bool one = false;
#pragma unroll
        for (uint32_t j = 0; j < PER; j++) {
            const uint32_t d = lane * PER + j;
            vals[j] = d < RADIX ? rowp[d] : 0u;
            local += vals[j];
            one |= vals[j] == len;
        }
        uint32_t incl = local;
#pragma unroll
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t up = __shfl_up(incl, off, 64);
            if (lane >= off)
                incl += up;
        }
        uint32_t run = coff[s] + incl - local;
        uint32_t* outp = lbase + ((size_t)p * seg_max + s) * RADIX;
#pragma unroll
        for (uint32_t j = 0; j < PER; j++) {
            const uint32_t d = lane * PER + j;
            if (d < RADIX)
                outp[d] = run;
            run += vals[j];
        }
        if (__ballot(one) != 0 && lane == 0)
            atomicAdd(&hdr->seg_trivial[p], 1u);
        return;
    }
    const uint64_t t = (uint64_t)(blockIdx.x - row_blocks) * blockDim.x + threadIdx.x;
    const uint32_t d = (uint32_t)(t % RADIX);
    const uint64_t pc = t / RADIX;
    const uint32_t c = (uint32_t)(pc % seg_chunks), p = (uint32_t)(pc / seg_chunks);
    if (p >= passes)
        return;
    const uint32_t s0 = c * kSegChunk, s1 = min(s0 + kSegChunk, nseg);
    uint32_t sum = 0;
    for (uint32_t s = s0; s < s1; s++)
        sum += lcnt[((size_t)p * seg_max + s) * RADIX + d];
    csum[((size_t)p * seg_chunks + c) * RADIX + d] = sum;
}

// One block: exclusive scan of the group sums over groups, per (pass,
// digit), in place; then per pass whether it is the identity for every
// segment (skipped), whether one digit holds over 1/16 of all segment nodes
// (rank by ballots), and the buffers.
template <int RB>
__global__ __launch_bounds__(1024) void k_lscan(uint32_t* __restrict__ csum, uint32_t passes,
                                                uint32_t seg_chunks, Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    __shared__ uint32_t s_skip[kMaxPasses];
    __shared__ uint32_t s_heavy[kMaxPasses];
    if (hdr->status != 0)
        return;
    const uint32_t nseg = hdr->n_segs, nodes = hdr->seg_nodes;
    const uint32_t used = (nseg + kSegChunk - 1) / kSegChunk;
    for (uint32_t p = threadIdx.x; p < passes; p += blockDim.x) {
        s_skip[p] = hdr->seg_trivial[p] == nseg ? 1u : 0u;
        s_heavy[p] = 0;
    }
    __syncthreads();
    for (uint32_t col = threadIdx.x; col < passes * RADIX; col += blockDim.x) {
        const uint32_t p = col / RADIX, d = col % RADIX;
        uint32_t* cp = csum + (size_t)p * seg_chunks * RADIX + d;
        uint32_t run = 0;
        for (uint32_t c = 0; c < used; c++) {
            const uint32_t v = cp[(size_t)c * RADIX];
            cp[(size_t)c * RADIX] = run;
            run += v;
        }
        if ((uint64_t)run * 16u > (uint64_t)nodes)
            atomicOr(&s_heavy[p], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t p = 0; p < passes; p++)
            hdr->sched[p].ballot = s_heavy[p];
        assign_kinds(s_skip, passes, hdr);
    }
}

// One thread per (pass, group, digit): subtract, for every segment of the
// group, the count of its digit in all segments before it.
template <int RB>
__global__ __launch_bounds__(256) void k_lfin(const uint32_t* __restrict__ lcnt,
                                              uint32_t* __restrict__ lbase,
                                              const uint32_t* __restrict__ csum, uint32_t passes,
                                              uint32_t seg_max, uint32_t seg_chunks, Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    if (hdr->status != 0)
        return;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t d = (uint32_t)(t % RADIX);
    const uint64_t pc = t / RADIX;
    const uint32_t c = (uint32_t)(pc % seg_chunks), p = (uint32_t)(pc / seg_chunks);
    if (p >= passes)
        return;
    const uint32_t nseg = hdr->n_segs;
    const uint32_t s0 = c * kSegChunk, s1 = min(s0 + kSegChunk, nseg);
    uint32_t run = csum[((size_t)p * seg_chunks + c) * RADIX + d];
    for (uint32_t s = s0; s < s1; s++) {
        const size_t at = ((size_t)p * seg_max + s) * RADIX + d;
        lbase[at] -= run;
        run += lcnt[at];
    }
}

// ---------------------------------------------------------------- relink
// Thread j, once the batch is known to be valid, at position j of the
// segments: next_out[order[j]] = order[j+1] inside the segment's range, NIL
// at its end; the segment's first node is its list's new head.  In the
// gather form results go to each list's own array in list-local indices.
__global__ __launch_bounds__(256) void k_frelink(OrderSrc src, ForestArgs F,
                                                 const uint32_t* __restrict__ ctable,
                                                 uint32_t* __restrict__ next_out,
                                                 uint32_t* __restrict__ new_heads,
                                                 const Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= hdr->seg_nodes)
        return;
    const SegMap sm{ctable, F.coff, nullptr};
    const uint32_t s = seg_of(sm, j, hdr->n_segs);
    const uint32_t l = F.segl[s];
    const uint32_t c1 = F.coff[s + 1];
    const uint32_t kind = hdr->final_kind;
    const uint32_t node = order_at(src, kind, j);
    const uint32_t succ = (j + 1 < c1) ? order_at(src, kind, j + 1) : kNil;
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    if (node < lo || node >= hi)
        return;  // cannot happen for a sorted batch; keeps every write in bounds
    if (F.next_out_ptrs) {
        ((uint32_t*)F.next_out_ptrs[l])[node - lo] = succ == kNil ? kNil : (uint32_t)(succ - lo);
        if (j == F.coff[s])
            new_heads[l] = (uint32_t)(node - lo);
    } else {
        next_out[node] = succ;
        if (j == F.coff[s])
            new_heads[l] = node;
    }
}

// One workgroup per list, once the batch is known to be valid: a short
// list's new links (sorted in LDS earlier) go to the caller's array in index
// order and its new head to new_heads; an empty list gets NIL.  Thread 0 of
// block 0 writes the batch status, valid or not.
__global__ __launch_bounds__(256) void k_fcommit(ForestArgs F, const uint32_t* __restrict__ snext,
                                                 const uint32_t* __restrict__ shead,
                                                 uint32_t* __restrict__ next_out,
                                                 uint32_t* __restrict__ new_heads,
                                                 int32_t* __restrict__ d_status, const Header* hdr)
{
    const int32_t st = hdr->status;
    const uint32_t l = blockIdx.x;
    if (l == 0 && threadIdx.x == 0)
        *d_status = st;
    if (st != 0 || l >= F.H || is_seg(F, l))
        return;
    const uint64_t lo = F.offsets[l], hi = F.offsets[l + 1];
    if (hi == lo) {
        if (threadIdx.x == 0)
            new_heads[l] = kNil;
        return;
    }
    const uint32_t len = (uint32_t)(hi - lo);
    if (F.next_out_ptrs) {
        uint32_t* out = (uint32_t*)F.next_out_ptrs[l];
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x)
            out[i] = snext[lo + i];
        if (threadIdx.x == 0)
            new_heads[l] = shead[l];
    } else {
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
            const uint32_t v = snext[lo + i];
            next_out[lo + i] = v == kNil ? kNil : v + (uint32_t)lo;
        }
        if (threadIdx.x == 0)
            new_heads[l] = shead[l] + (uint32_t)lo;
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

template <typename KeyT, int RB, class Src>
static hipError_t launch_fpack(const Plan& P, const Src& src, const ForestArgs& F, char* ws,
                               hipStream_t s)
{
    const uint32_t blocks = (uint32_t)((P.n + P.pack_chunk - 1) / P.pack_chunk);
    const size_t shm = (size_t)kPackSlots * P.passes * P.radix * sizeof(uint32_t);
    hipLaunchKernelGGL((k_fpack<KeyT, RB, Src>), dim3(blocks), dim3(256), shm, s, src, F,
                       P.pack_chunk, key_float_sel<KeyT>(P.flags), key_xor_mask<KeyT>(P.flags),
                       P.passes, P.seg_max, (NodeRec<KeyT>*)(ws + P.o_nodes),
                       (uint32_t*)(ws + P.o_lcnt), (Header*)(ws + P.o_header));
    return hipGetLastError();
}

template <typename KeyT, int RB, int CUT>
static hipError_t launch_fsmall_cut(const Plan& P, const ForestArgs& F, const uint32_t* next_in,
                                    const void* keys, char* ws, hipStream_t s)
{
    hipLaunchKernelGGL((k_fsmall<KeyT, RB, CUT>), dim3(P.num_lists), dim3(kSmallThreads), 0, s,
                       F, next_in, (const KeyT*)keys, key_float_sel<KeyT>(P.flags),
                       key_xor_mask<KeyT>(P.flags), P.passes, (uint32_t*)(ws + P.o_snext),
                       (uint32_t*)(ws + P.o_shead), (Header*)(ws + P.o_header));
    return hipGetLastError();
}

template <typename KeyT, int RB>
static hipError_t launch_rb(const Plan& P, const ForestArgs& F, const uint32_t* next_in,
                            const void* keys, char* ws, hipStream_t s, Prof* prof)
{
    constexpr uint32_t RADIX = 1u << RB;
    hipError_t e;
    Header* hdr = (Header*)(ws + P.o_header);
    // short lists, in LDS
    mark(prof, s, kStageSmall);
    if (P.cutoff <= 1024)
        e = launch_fsmall_cut<KeyT, RB, 1024>(P, F, next_in, keys, ws, s);
    else if (P.cutoff <= 2048)
        e = launch_fsmall_cut<KeyT, RB, 2048>(P, F, next_in, keys, ws, s);
    else
        e = launch_fsmall_cut<KeyT, RB, 4096>(P, F, next_in, keys, ws, s);
    if (e != hipSuccess)
        return e;
    // segments: pack with per-list counts
    mark(prof, s, kStagePack);
    if (F.next_in_ptrs)
        e = launch_fpack<KeyT, RB>(P, GatherSrc<KeyT>{F.lm, F.next_in_ptrs, F.key_ptrs}, F, ws, s);
    else
        e = launch_fpack<KeyT, RB>(P, DirectSrc<KeyT>{next_in, (const KeyT*)keys}, F, ws, s);
    if (e != hipSuccess)
        return e;
    // per-list digit bases
    mark(prof, s, kStageBases);
    {
        const uint32_t row_blocks = (uint32_t)(((uint64_t)P.passes * P.seg_max + 3) / 4);
        const uint64_t col_threads = (uint64_t)P.passes * P.seg_chunks * RADIX;
        const uint32_t col_blocks = (uint32_t)((col_threads + 255) / 256);
        hipLaunchKernelGGL((k_lprep<RB>), dim3(row_blocks + col_blocks), dim3(256), 0, s,
                           (const uint32_t*)(ws + P.o_lcnt), (uint32_t*)(ws + P.o_lbase),
                           (uint32_t*)(ws + P.o_csum), (const uint32_t*)(ws + P.o_coff), P.passes,
                           P.seg_max, P.seg_chunks, row_blocks, hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL((k_lscan<RB>), dim3(1), dim3(1024), 0, s, (uint32_t*)(ws + P.o_csum),
                           P.passes, P.seg_chunks, hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL((k_lfin<RB>), dim3(col_blocks), dim3(256), 0, s,
                           (const uint32_t*)(ws + P.o_lcnt), (uint32_t*)(ws + P.o_lbase),
                           (const uint32_t*)(ws + P.o_csum), P.passes, P.seg_max, P.seg_chunks,
                           hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    // ranking of the segments as a forest
    mark(prof, s, kStageWalk0);
    if ((e = launch_fwalk0<KeyT>(P, F, ws, s)) != hipSuccess)
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
    if ((e = launch_unchain<KeyT>(P, ws, s, prof)) != hipSuccess)
        return e;
    if (P.look64)
        e = launch_passes<KeyT, uint64_t, true>(P, ws, s, prof, true);
    else
        e = launch_passes<KeyT, uint32_t, true>(P, ws, s, prof, true);
    return e;
}

template <typename KeyT>
static hipError_t launch_key(const Plan& P, const ForestArgs& F, const uint32_t* next_in,
                             const void* keys, char* ws, hipStream_t s, Prof* prof)
{
    switch (P.RB) {
    case 1: return launch_rb<KeyT, 1>(P, F, next_in, keys, ws, s, prof);
    case 2: return launch_rb<KeyT, 2>(P, F, next_in, keys, ws, s, prof);
    case 4: return launch_rb<KeyT, 4>(P, F, next_in, keys, ws, s, prof);
    default: return launch_rb<KeyT, 8>(P, F, next_in, keys, ws, s, prof);
    }
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
    F.cutoff = P.cutoff;
    F.lm.table = (const uint32_t*)(ws + P.o_table);
    F.lm.offsets = offsets;
    F.lm.num_lists = P.num_lists;
    F.lm.log_block = P.log_block;
    F.head_bits = (const uint32_t*)(ws + P.o_headbits);
    F.lrank = (const uint32_t*)(ws + P.o_lseg);
    F.segl = (const uint32_t*)(ws + P.o_segl);
    F.coff = (const uint32_t*)(ws + P.o_coff);
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
    mark(prof, s, kStagePlan);
    hipLaunchKernelGGL(k_fplan, dim3(1), dim3(1024), 0, s, F, (uint32_t*)(ws + P.o_lseg),
                       (uint32_t*)(ws + P.o_segl), (uint32_t*)(ws + P.o_coff),
                       (uint32_t*)(ws + P.o_headbits), hdr);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_ftables, dim3(P.num_lists), dim3(256), 0, s, F,
                       (uint32_t*)(ws + P.o_table), (uint32_t*)(ws + P.o_ctable), hdr);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    switch (P.key_bytes) {
    case 1: e = launch_key<uint8_t>(P, F, next_in, keys, ws, s, prof); break;
    case 2: e = launch_key<uint16_t>(P, F, next_in, keys, ws, s, prof); break;
    case 4: e = launch_key<uint32_t>(P, F, next_in, keys, ws, s, prof); break;
    default: e = launch_key<uint64_t>(P, F, next_in, keys, ws, s, prof); break;
    }
    if (e != hipSuccess)
        return e;
    {
        mark(prof, s, kStageRelink);
        const OrderSrc src = P.key_bytes == 8 ? order_src<uint64_t>(P, ws) : order_src<uint32_t>(P, ws);
        hipLaunchKernelGGL(k_frelink, dim3((uint32_t)((P.n + 255) / 256)), dim3(256), 0, s, src, F,
                           (const uint32_t*)(ws + P.o_ctable), next_out, new_heads,
                           (const Header*)hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        mark(prof, s, kStageCommit);
        hipLaunchKernelGGL(k_fcommit, dim3(P.num_lists), dim3(256), 0, s, F,
                           (const uint32_t*)(ws + P.o_snext), (const uint32_t*)(ws + P.o_shead),
                           next_out, new_heads, d_status, (const Header*)hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    mark(prof, s, kStageCount);
    return hipSuccess;
}

}  // namespace pbit
