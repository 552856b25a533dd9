// Device code shared by the single-list path (pbit_kernels.hip) and the
// many-list path (pbit_forest.hip): node records, hashing, the pack kernel,
// chain unloading, the pass schedule and the stable digit pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pbit.h"
#include "pbit_internal.h"

namespace pbit {

// ---------------------------------------------------------------- records
// Packed node record: next and key in one load (8 bytes, 16 for u64 keys).
template <typename KeyT> struct NodeRec { uint32_t next; uint32_t key; };
template <> struct __attribute__((aligned(16))) NodeRec<uint64_t> { uint32_t next; uint32_t pad; uint64_t key; };

// (key, node) entry of a level-0 chain.
template <typename KeyT> struct Entry { uint32_t key; uint32_t idx; };
template <> struct __attribute__((aligned(16))) Entry<uint64_t> { uint64_t key; uint32_t idx; uint32_t pad; };

template <typename KeyT> __device__ __forceinline__ KeyT entry_key(const Entry<KeyT>& e) { return (KeyT)e.key; }

// Level-0 chain slots, planar: entry t of chain c sits in plane t / kPlane at
// chain c's block of kPlane entries, so the first kPlane entries of all chains
// (where most chains end: their mean length is 2^kLog0) are one dense array
// that the walk fills and unchain reads nearly in order.
#ifndef PBIT_PLANE
#define PBIT_PLANE 16
#endif
constexpr uint32_t kPlane = PBIT_PLANE;
__device__ __forceinline__ size_t ent_at(uint32_t n_chains, uint32_t c, uint32_t t)
{
    return (size_t)(t / kPlane) * ((size_t)n_chains * kPlane) + (size_t)c * kPlane + (t % kPlane);
}

// (key, node) pair of the list-order buffers the digit passes stream through:
// one 8-byte (16-byte for 64-bit keys) record per element, so a pass reads and
// writes one contiguous run per digit instead of two half-length runs.
// Narrow keys widen to 32 bits; a 64-bit key is kept as two words, so its
// pair is 12 bytes (three-word loads and stores) rather than a padded 16.
template <typename KeyT> struct __attribute__((aligned(8))) Pair { uint32_t key; uint32_t idx; };
template <> struct Pair<uint64_t> { uint32_t klo; uint32_t khi; uint32_t idx; };

template <typename KeyT> __device__ __forceinline__ Pair<KeyT> make_pair_kv(KeyT k, uint32_t i)
{
    Pair<KeyT> p;
    if constexpr (sizeof(KeyT) == 8) {
        p.klo = (uint32_t)k;
        p.khi = (uint32_t)((uint64_t)k >> 32);
    } else {
        p.key = k;
    }
    p.idx = i;
    return p;
}

template <typename KeyT> __device__ __forceinline__ KeyT pair_key(const Pair<KeyT>& p)
{
    if constexpr (sizeof(KeyT) == 8)
        return ((uint64_t)p.khi << 32) | p.klo;
    else
        return (KeyT)p.key;
}

// Where the sorted order ends up: the idx field of pairs A, or an index buffer.
struct OrderSrc {
    const uint32_t* pair_idx;  // &pairsA[0].idx
    uint32_t pair_words;       // pair stride in 32-bit words
    const uint32_t* idxA;
    const uint32_t* idxB;
};
__device__ __forceinline__ uint32_t order_at(const OrderSrc& o, uint32_t kind, uint64_t j)
{
    if (kind == kBufIdxA)
        return o.idxA[j];
    if (kind == kBufIdxB)
        return o.idxB[j];
    return o.pair_idx[j * o.pair_words];
}

// Entries of a level-0 chain a walker gathers in registers before storing them.
template <typename KeyT> struct SegLen {
    static constexpr uint32_t value = sizeof(KeyT) == 8 ? PBIT_SEGLEN / 2 : PBIT_SEGLEN;
};

// Digit-pass tile shape (block threads x items per thread), the same for
// every pattern width.  The pass is latency-bound, so the shape is chosen for
// resident waves:
//  - Keys of up to 32 bits: 1024 x 6 = 6144 elements.  The block needs
//    68.6 KB of LDS and at most 64 VGPRs (8 waves per SIMD), so two blocks
//    share a CU: 32 waves, each ranking while others wait on HBM.  (768 x 8,
//    the same tile at 24 waves per CU, was 6 % slower; 1024 x 5 and 896 x 6
//    slower still.)
//  - 64-bit keys: 1024 x 8.  The 16-byte staging slots make the LDS tile
//    128 KB, one block per CU whatever its width, so the widest block wins.
// `waves` is the occupancy the kernel is compiled for (waves per SIMD),
// which caps its registers.
template <typename KeyT, int RB> struct PassShape {
    static constexpr int block = 1024;
    static constexpr int items = sizeof(KeyT) == 8 ? 8 : 6;
    static constexpr int waves = sizeof(KeyT) == 8 ? 4 : 8;
};

// Consecutive tiles given to one XCD in a row (default tile order).
// Work-groups go to the 8 XCDs round-robin by block index, so block b takes
// tile (q / C) * 8C + (b % 8) * C + q % C, q = b / 8, C = kPassChunk: each
// XCD then writes C neighbouring tiles' runs of every digit, and the partial
// cache lines where two tiles' runs meet merge in that XCD's L2 instead of
// being written back twice (with 8-bit patterns a tile's runs average 24
// elements, so most of its writes touch such lines: 11 % of the pass time at
// 2^24 keys).  The look-back follows tile order, so the first tile of a chunk
// waits on a tile that starts 8(C-1) blocks later.  When other kernels share
// the device they can hold the XCDs such a tile needs; calls that expect that
// take tiles from a ticket counter in block start order instead (PBIT_SHARED),
// which never waits on a tile that has not started.
#ifndef PBIT_PASS_CHUNK
#define PBIT_PASS_CHUNK 16
#endif
constexpr uint32_t kPassChunk = PBIT_PASS_CHUNK;

__device__ __forceinline__ void set_error(int32_t* status, int32_t code)
{
    atomicCAS(status, 0, code);
}

template <typename T> __device__ __forceinline__ T ld_agent(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> __device__ __forceinline__ void st_agent(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------- init
static __global__ void k_zero(uint32_t* __restrict__ p, size_t words)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride)
        p[i] = 0u;
}

// ---------------------------------------------------------------- hashing
// In-degree check: over a valid list (or set of lists) the non-NIL next[]
// values are every node except the heads, each once.  The sum of a 64-bit
// mixing hash over them must equal the sum over all nodes minus the heads.
__device__ __forceinline__ uint64_t mix64(uint64_t x, uint64_t k)
{
    x ^= x >> 31;
    x *= k;
    x ^= x >> 29;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 32;
    return x;
}
constexpr uint64_t kHashK1 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kHashK2 = 0xD6E8FEB86659FD93ull;

// ---------------------------------------------------------------- pack
// Where pack reads node i: one pair of next[]/keys[] arrays over all nodes...
template <typename KeyT> struct DirectSrc {
    const uint32_t* next;
    const KeyT* keys;
    __device__ __forceinline__ void load(size_t i, uint32_t n, uint32_t& nx, KeyT& k,
                                         bool& bad) const
    {
        nx = next[i];
        k = keys[i];
        bad |= (nx != kNil) && (nx >= n);
    }
};

// ... or records of `stride` bytes (the paper's node structure, Sec. 2: the
// link and the data side by side): node i's next index is the uint32 at byte
// next_off of record i, its key the KeyT at byte key_off.
template <typename KeyT> struct AosSrc {
    const char* base;
    uint64_t stride;
    uint32_t next_off;
    uint32_t key_off;
    __device__ __forceinline__ void load(size_t i, uint32_t n, uint32_t& nx, KeyT& k,
                                         bool& bad) const
    {
        const char* r = base + (uint64_t)i * stride;
        nx = *(const uint32_t*)(r + next_off);
        k = *(const KeyT*)(r + key_off);
        bad |= (nx != kNil) && (nx >= n);
    }
};

// Node -> list of a many-list sort: lists own contiguous node ranges
// [offsets[l], offsets[l+1]); table[b] is the list holding node b << log_block.
struct LidMap {
    const uint32_t* table;
    const uint64_t* offsets;
    uint32_t num_lists;
    uint32_t log_block;
};

__device__ __forceinline__ uint32_t list_of(const LidMap& lm, uint32_t node)
{
    uint32_t l = min(lm.table[node >> lm.log_block], lm.num_lists - 1u);
    while (l + 1 < lm.num_lists && lm.offsets[l + 1] <= node)
        l++;
    return l;
}

// ... or one array pair per list (device pointers), holding list-local node
// indices; node i of the batch is node i - offsets[l] of list l.
template <typename KeyT> struct GatherSrc {
    LidMap lm;
    const uint64_t* next_ptrs;
    const uint64_t* key_ptrs;
    __device__ __forceinline__ void load(size_t i, uint32_t, uint32_t& nx, KeyT& k,
                                         bool& bad) const
    {
        const uint32_t l = list_of(lm, (uint32_t)i);
        const uint64_t off = lm.offsets[l];
        const uint64_t len = lm.offsets[l + 1] - off;
        const uint64_t loc = i - off;
        if (i < off || loc >= len) {
            // the node -> list table does not cover node i: the batch is not
            // what k_fprep validated, so flag it instead of reading
            nx = kNil;
            k = 0;
            bad = true;
            return;
        }
        const uint32_t nl = ((const uint32_t*)next_ptrs[l])[loc];
        k = ((const KeyT*)key_ptrs[l])[loc];
        if (nl == kNil) {
            nx = kNil;
        } else if (nl < len) {
            nx = (uint32_t)(nl + off);
        } else {
            nx = kNil;
            bad = true;
        }
    }
};

// The order-preserving key transform of the flags.  Floating-point keys
// (sign-magnitude): a negative pattern is inverted whole, a non-negative one
// gets its sign bit set, so unsigned order of the result is the numeric order
// (float_sel is all ones or zero).  Then the XOR mask: the sign bit for
// two's-complement keys, all bits for descending order.
template <typename KeyT>
__device__ __forceinline__ KeyT transform_key(KeyT k, KeyT float_sel, KeyT xor_mask)
{
    constexpr uint32_t W = sizeof(KeyT) * 8;
    const KeyT neg = (KeyT)((KeyT)0 - (KeyT)(k >> (W - 1)));
    k ^= (KeyT)((KeyT)(neg | (KeyT)((KeyT)1 << (W - 1))) & float_sel);
    return (KeyT)(k ^ xor_mask);
}

// Sources whose next[] and keys[] can be read four nodes at a time with
// 16-byte loads (when both arrays are 16-byte aligned).
template <class Src> struct Loads4 { static constexpr bool value = false; };
template <> struct Loads4<DirectSrc<uint32_t>> { static constexpr bool value = true; };

// Node records, the count of every pattern value of every key pass, the NIL
// count and the hash sums sum h(next) - sum h(i).
template <typename KeyT, int RB, class Src>
__global__ __launch_bounds__(256) void k_pack(Src src, uint32_t n, KeyT float_sel, KeyT xor_mask,
                                              uint32_t passes,
                                              NodeRec<KeyT>* __restrict__ nodes,
                                              uint32_t* __restrict__ hist, Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    extern __shared__ uint32_t s_hist[];  // passes * RADIX
    // a batch whose slabs or heads failed validation is not read at all (the
    // node -> list table of a gather batch is incomplete then)
    if (__syncthreads_or(hdr->status != 0))
        return;
    const uint32_t nbins = passes * RADIX;
    for (uint32_t i = threadIdx.x; i < nbins; i += blockDim.x)
        s_hist[i] = 0;
    __syncthreads();
    bool bad = false;
    uint64_t h1 = 0, h2 = 0;
    uint32_t nils = 0;
    // one node: key transform, hashes, NIL count, histograms; returns the
    // transformed key (the caller writes the record)
    auto take = [&](size_t i, uint32_t nx, KeyT k) -> KeyT {
        k = transform_key<KeyT>(k, float_sel, xor_mask);
        if (nx == kNil) {
            nils++;
        } else {
            h1 += mix64(nx + 1ull, kHashK1);
            h2 += mix64(nx + 1ull, kHashK2);
        }
        h1 -= mix64(i + 1ull, kHashK1);
        h2 -= mix64(i + 1ull, kHashK2);
        for (uint32_t p = 0; p < passes; p++) {
            const uint32_t d = (uint32_t)(k >> (p * RB)) & (RADIX - 1u);
            atomicAdd(&s_hist[p * RADIX + d], 1u);
        }
        return k;
    };
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t gid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t first = 0;  // nodes below this index were taken four at a time
    if constexpr (Loads4<Src>::value) {
        if ((((uintptr_t)src.next | (uintptr_t)src.keys) & 15u) == 0) {
            const size_t quads = n / 4;
            for (size_t q = gid; q < quads; q += stride) {
                const uint4 a = ((const uint4*)src.next)[q];
                const uint4 b = ((const uint4*)src.keys)[q];
                const uint32_t nx[4] = {a.x, a.y, a.z, a.w};
                uint32_t k[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    bad |= (nx[j] != kNil) && (nx[j] >= n);
                    k[j] = take(4 * q + j, nx[j], k[j]);
                }
                uint4* out = (uint4*)(nodes + 4 * q);
                out[0] = make_uint4(nx[0], k[0], nx[1], k[1]);
                out[1] = make_uint4(nx[2], k[2], nx[3], k[3]);
            }
            first = quads * 4;
        }
    }
    for (size_t i = first + gid; i < n; i += stride) {
        uint32_t nx;
        KeyT k;
        src.load(i, n, nx, k, bad);
        k = take(i, nx, k);
        NodeRec<KeyT> r;
        r.next = nx;
        r.key = k;
        if constexpr (sizeof(KeyT) == 8) r.pad = 0;
        nodes[i] = r;
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
    const uint32_t wave = threadIdx.x / 64;
    if (__lane_id() == 0) {
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
        atomicAdd((unsigned long long*)&hdr->hsum[0], (unsigned long long)a);
        atomicAdd((unsigned long long*)&hdr->hsum[1], (unsigned long long)b);
        if (z)
            atomicAdd(&hdr->nil_count, z);
    }
    for (uint32_t i = threadIdx.x; i < nbins; i += blockDim.x) {
        const uint32_t v = s_hist[i];
        if (v)
            atomicAdd(&hist[i], v);
    }
}

// ---------------------------------------------------------------- unchain
// Every level-0 chain to list order: its stored entries (up to `cap`) are
// copied to its place, 2^kLog0 threads (the mean chain length) per chain.
// A chain longer than its slot also needs the rest re-walked from its resume
// node, one dependent load per node.  The first kLongListMax such chains are
// listed by the walk and taken by the first kLongBlocks blocks, which are
// dispatched first, so that latency-bound tail overlaps the copy; any further
// ones (many when the slot is short) are walked by their own chain's first
// thread.
constexpr uint32_t kLongBlocks = kLongListMax / 256;
constexpr uint32_t kUnchainThreads = 1u << kLog0;
// Entries one unchain thread copies per step: two 8-byte entries (one 16-byte
// load) for keys of up to 32 bits, one 16-byte entry for 64-bit keys.  (Two
// beat one by 22 % and four by 16 %.)
template <typename KeyT> struct UnchainPer { static constexpr uint32_t value = sizeof(KeyT) == 8 ? 1 : 2; };

// End of a level-0 walk: where the rest of a long chain is walked from.
// long_list holds {chain, resume node} pairs for the early blocks; resume[c]
// is the node for the chain's own group, or kNil.
__device__ __forceinline__ void record_long_chain(uint32_t c, uint32_t len, uint32_t cap,
                                                  uint32_t rest_from, uint32_t* resume,
                                                  uint32_t* long_list, Header* hdr)
{
    uint32_t own = kNil;
    if (len > cap) {
        const uint32_t k = atomicAdd(&hdr->n_long, 1u);
        if (k < kLongListMax) {
            long_list[2 * k] = c;
            long_list[2 * k + 1] = rest_from;
        } else {
            own = rest_from;
        }
    }
    resume[c] = own;
}

// Write the rest of chain c (positions cap..len-1 of the chain) from node cur.
template <typename KeyT>
__device__ __forceinline__ void walk_rest(const NodeRec<KeyT>* __restrict__ nodes, uint32_t cur,
                                          uint64_t pos, uint64_t end, uint32_t n,
                                          Pair<KeyT>* __restrict__ out)
{
    while (pos < end && cur < n) {
        const NodeRec<KeyT> r = nodes[cur];
        out[pos] = make_pair_kv<KeyT>((KeyT)r.key, cur);
        pos++;
        cur = r.next;
    }
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_unchain(const uint2* __restrict__ chain_rec,
                                                 const Entry<KeyT>* __restrict__ ent,
                                                 uint32_t n_chains, uint32_t cap,
                                                 const uint32_t* __restrict__ offn_chain, uint32_t n,
                                                 const NodeRec<KeyT>* __restrict__ nodes,
                                                 const uint32_t* __restrict__ resume,
                                                 const uint32_t* __restrict__ long_list,
                                                 Pair<KeyT>* __restrict__ out, Header* hdr)
{
    constexpr uint32_t PER = UnchainPer<KeyT>::value;
    // threads per chain: together they copy the mean chain length per step
    constexpr uint32_t G = kUnchainThreads / PER;
    static_assert(kUnchainThreads <= kPlane, "a chain's first copy round lies in its first plane");
    if (blockIdx.x < kLongBlocks) {
        if (hdr->status != 0)
            return;
        const uint32_t listed = min(hdr->n_long, kLongListMax);
        const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
        if (i < listed) {
            const uint32_t c = long_list[2 * i];
            if (c < n_chains) {
                const uint64_t base = offn_chain[c];
                walk_rest<KeyT>(nodes, long_list[2 * i + 1], base + cap,
                                min<uint64_t>(base + chain_rec[c].y, (uint64_t)n), n, out);
            }
        }
        return;
    }
    const uint64_t g = (blockIdx.x - kLongBlocks) * (uint64_t)blockDim.x + threadIdx.x;
    const uint32_t c = (uint32_t)(g / G);
    if (c >= n_chains)
        return;
    const uint32_t lead = (uint32_t)(g % G);
    const uint32_t t0 = lead * PER;
    // the chain's record, its offset and its first entries are loaded
    // together, before the status is known: every chain's slot holds its
    // first plane, so the addresses are valid whatever was stored there
    const int32_t st = hdr->status;
    const uint2 cr = chain_rec[c];
    const uint32_t base = offn_chain[c];
    uint4 v0[PER > 1 ? PER / 2 : 1];
    Entry<KeyT> e0;
    if constexpr (PER > 1) {
        const uint4* src = (const uint4*)&ent[ent_at(n_chains, c, t0)];
#pragma unroll
        for (uint32_t h = 0; h < PER / 2; h++)
            v0[h] = src[h];
    } else {
        e0 = ent[ent_at(n_chains, c, t0)];
    }
    if (st != 0)
        return;
    const uint32_t full = cr.y;
    const uint32_t len = min(full, cap);
    if (lead == 0 && full > cap) {
        const uint32_t own = resume[c];
        if (own != kNil)
            walk_rest<KeyT>(nodes, own, (uint64_t)base + cap,
                            min<uint64_t>((uint64_t)base + full, (uint64_t)n), n, out);
    }
    // entries t .. t + PER - 1 (adjacent in one plane, t a multiple of PER)
    // to list positions base + t ..
    auto put = [&](uint32_t t, const uint4* v, const Entry<KeyT>& e) {
        const uint32_t pos = base + t;
        if constexpr (PER > 1) {
#pragma unroll
            for (uint32_t j = 0; j < PER; j++) {
                const uint4 w = v[j / 2];
                const uint32_t key = (j & 1) ? w.z : w.x, idx = (j & 1) ? w.w : w.y;
                if (j == 0 || (t + j < len && pos + j < n))
                    out[pos + j] = make_pair_kv<KeyT>((KeyT)key, idx);
            }
        } else {
            out[pos] = make_pair_kv<KeyT>(entry_key<KeyT>(e), e.idx);
        }
    };
    if (t0 >= len || base + t0 >= n)
        return;
    put(t0, v0, e0);
    for (uint32_t t = t0 + kUnchainThreads; t < len; t += kUnchainThreads) {
        if (base + t >= n)
            break;
        uint4 v[PER > 1 ? PER / 2 : 1];
        Entry<KeyT> e;
        if constexpr (PER > 1) {
            const uint4* src = (const uint4*)&ent[ent_at(n_chains, c, t)];
#pragma unroll
            for (uint32_t h = 0; h < PER / 2; h++)
                v[h] = src[h];
        } else {
            e = ent[ent_at(n_chains, c, t)];
        }
        put(t, v, e);
    }
}

// ---------------------------------------------------------------- schedule
// Buffers of each pass: the list order starts as (key, node) pairs A; passes
// go pairs to pairs in ping-pong, and the last pass that runs writes node
// indices only.  Skipped passes (the identity) leave the buffers as they are.
// The last pass needs only its own digit of each key (the patterns below it
// are already in the order, those above it are constant), so with `packable`
// (node indices below 2^(32 - rb)) the pass before it writes one word per
// element, that digit over the node index, instead of a pair.  For one list
// of 64-bit keys, passes from `hi_from` on (the high 32 key bits) run as
// 32-bit-key passes over (high half, node) pairs, which the last running
// pass before them writes.
// The buffer of each pass (in, out, and the packed digit's position) from
// the passes that run, handed to emit(p, in, out, pk_shift); returns the
// buffer holding the sorted order.  Also used on the host, with no pass
// skipped, for the buffer a pass can expect before it reads the schedule.
template <class Emit>
__host__ __device__ inline uint32_t pass_kinds(const uint32_t* skip, uint32_t passes,
                                               bool packable, uint32_t rb, uint32_t hi_from,
                                               Emit emit)
{
    int last = -1, prev = -1;
    for (uint32_t p = 0; p < passes; p++)
        if (!skip[p]) {
            prev = last;
            last = (int)p;
        }
    const bool packed = packable && prev >= 0;
    uint32_t cur = kBufPairsA;
    for (uint32_t p = 0; p < passes; p++) {
        uint32_t pk_shift = 0;
        // the next pass that runs after p
        int next = -1;
        for (uint32_t q = p + 1; q < passes && next < 0; q++)
            if (!skip[q])
                next = (int)q;
        const bool b = !buf_in_b(cur);  // the other buffer
        uint32_t out;
        if ((int)p == last) {
            out = kBufIdxA;
        } else if (packed && (int)p == prev) {
            out = b ? kBufPackB : kBufPackA;
            // the digit's bit position in the writer's own key (a high-half
            // pass holds key bits 32.. only)
            pk_shift = (uint32_t)last * rb - (p >= hi_from ? 32u : 0u);
        } else if (next >= (int)hi_from) {
            out = b ? kBufHalfB : kBufHalfA;
        } else {
            out = b ? kBufPairsB : kBufPairsA;
        }
        emit(p, cur, out, pk_shift);
        if (!skip[p])
            cur = out;
    }
    return cur;
}

__device__ __forceinline__ void assign_kinds(const uint32_t* skip, uint32_t passes, Header* hdr,
                                             bool packable = false, uint32_t rb = 0,
                                             uint32_t hi_from = kMaxPasses)
{
    hdr->final_kind = pass_kinds(skip, passes, packable, rb, hi_from,
                                 [&](uint32_t p, uint32_t in, uint32_t out, uint32_t pk) {
                                     PassSched ps = hdr->sched[p];
                                     ps.skip = skip[p];
                                     ps.in_kind = in;
                                     ps.out_kind = out;
                                     ps.pk_shift = pk;
                                     hdr->sched[p] = ps;
                                 });
}

// Per pass (one list): exclusive scan of the digit counts (global digit
// bases), whether the pass is the identity (every element has the same
// digit: the paper's empty groups), whether one digit is frequent enough to
// rank by ballots, and the buffers.  A block-level routine (256 threads,
// radix <= 256): one extra block of the level-0 walk.
__device__ __forceinline__ void schedule_body(const uint32_t* __restrict__ hist,
                                              uint32_t* __restrict__ dbase, uint32_t passes,
                                              uint32_t n, uint32_t radix, Header* hdr,
                                              uint32_t hi_from)
{
    __shared__ uint32_t s_v[256];
    __shared__ uint32_t s_skip[kMaxPasses];
    const uint32_t tid = threadIdx.x;
    for (uint32_t p = 0; p < passes; p++) {
        uint32_t v = 0;
        if (tid < radix) {
            v = hist[p * radix + tid];
            s_v[tid] = v;
        }
        __syncthreads();
        const int full = (tid < radix) && (v == n);
        const int any_full = __syncthreads_or(full);
        // a digit holding over 1/16 of the elements makes many lanes of a
        // wave share one LDS mask word; such passes rank by ballots instead
        const int heavy = (tid < radix) && ((uint64_t)v * 16u > (uint64_t)n);
        const int any_heavy = __syncthreads_or(heavy);
        if (tid == 0) {
            uint32_t sum = 0;
            for (uint32_t d = 0; d < radix; d++) {
                const uint32_t x = s_v[d];
                s_v[d] = sum;
                sum += x;
            }
            s_skip[p] = any_full ? 1u : 0u;
            hdr->sched[p].ballot = any_heavy ? 1u : 0u;
        }
        __syncthreads();
        if (tid < radix)
            dbase[p * radix + tid] = s_v[tid];
        __syncthreads();
    }
    if (tid == 0) {
        const uint32_t rb = 31u - (uint32_t)__clz(radix);
        assign_kinds(s_skip, passes, hdr, (uint64_t)n <= (1ull << (32 - rb)), rb, hi_from);
    }
}

template <int RB>
__global__ __launch_bounds__(256) void k_schedule(const uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ dbase, uint32_t passes,
                                                  uint32_t n, Header* hdr, uint32_t hi_from)
{
    schedule_body(hist, dbase, passes, n, 1u << RB, hdr, hi_from);
}

// ---------------------------------------------------------------- segments
// Many lists sorted together: the lists' elements sit in one array of
// positions, list s at [coff[s], coff[s+1]) (segments, in list order).
// table[b] is the segment holding position b << kSegLog; lbase is a pass's
// per-segment digit base table ([segment][radix], see the digit pass).
struct SegMap {
    const uint32_t* table;
    const uint32_t* coff;
    const uint32_t* lbase;
};

__device__ __forceinline__ uint32_t seg_of(const SegMap& sm, uint32_t pos, uint32_t nseg)
{
    uint32_t s = min(sm.table[pos >> kSegLog], nseg - 1u);
    while (s + 1 < nseg && sm.coff[s + 1] <= pos)
        s++;
    return s;
}

// Segments one digit-pass tile may span: a tile holds at most 8192 elements
// and every segment more than kMinSegLen, so at most 8192 / 1025 + 2 = 9.
constexpr uint32_t kTileSegs = 16;

// ---------------------------------------------------------------- digit pass
// One stable split on the pattern at bit `shift`.  A tile of BLOCK * ITEMS
// consecutive list positions is loaded wave-striped and ranked per wave: an item's peers (the lanes whose
// item has the same digit) come from a per-wave LDS lane mask per digit (or,
// when one digit is frequent enough to make lanes queue on one mask word,
// from K ballots, as the schedule decides per pass); the
// first lane of each peer group adds the group size to a wave-private LDS
// counter (items in program order) and its peers take the returned base from
// it.  Counts are scanned across waves, tiles are chained by decoupled
// look-back (Merrill & Garland), and the tile is staged in LDS grouped by
// digit and written out in runs.  Tiles go to blocks in XCD chunks (see
// kPassChunk) or, with `ticket`, in block start order from a per-pass
// counter.  The look-back spin is bounded: a tile that waits too long on a
// predecessor counts that predecessor's digit in its input itself.
//
// An element's destination is base + P_d(j), where P_d(j) is the number of
// elements before position j with the same digit d (local rank plus the
// look-back prefix).  For one list the base is the digit's global start
// dbase[d].  For many lists in segments (SEG), each list must stay in its own
// range: list s's element with digit d goes to
//   coff[s] + #(list s elements with digit < d) + #(list s elements with
//   digit d before it)
// = lbase[s][d] + P_d(j), with lbase[s][d] = coff[s] + (digit-d exclusive
// count inside list s) - P_d(coff[s]) (wrapping 32-bit arithmetic), built
// from per-list digit counts before the passes.
//
// LW is the look-back word: 2 flag bits over a 30-bit count (uint32_t, for
// n < 2^30) or 2 flag bits over a 32-bit count (uint64_t).
template <typename LW> struct Look;
template <> struct Look<uint32_t> {
    static constexpr uint32_t AGG = 1u << 30, PREFIX = 2u << 30, MASK = (1u << 30) - 1u;
};
template <> struct Look<uint64_t> {
    static constexpr uint64_t AGG = 1ull << 32, PREFIX = 2ull << 32, MASK = 0xFFFFFFFFull;
};

template <typename SKey> struct KV { SKey key; uint32_t idx; };

// Look-back words read per round trip by a digit's thread.
#ifndef PBIT_LOOK_WINDOW
#define PBIT_LOOK_WINDOW 4
#endif
constexpr uint32_t kLookWindow = PBIT_LOOK_WINDOW;

// HI: a pass over the high 32 bits of one list's 64-bit keys, run as a
// 32-bit-key pass (KeyT = uint32_t, `shift` relative to bit 32); its input may
// still be the full (key, node) pairs when no pass over the low half ran.
template <typename KeyT, int RB, int BLOCK, int ITEMS, typename LW, bool SEG, bool HI = false>
__global__ __launch_bounds__(BLOCK, (PassShape<KeyT, RB>::waves)) void k_digit_pass(
    uint32_t pass, uint32_t shift, uint32_t n_all, Pair<KeyT>* __restrict__ pairsA,
    Pair<KeyT>* __restrict__ pairsB, uint32_t* __restrict__ idxA, uint32_t* __restrict__ idxB,
    const uint32_t* __restrict__ dbase, LW* __restrict__ look, Header* hdr, SegMap sm,
    uint32_t spin_limit, uint32_t ticket, uint32_t exp_in)
{
    using LK = Look<LW>;
    constexpr uint32_t RADIX = 1u << RB;
    constexpr uint32_t WAVES = BLOCK / 64;
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint32_t s_wave[WAVES][RADIX];
    __shared__ uint32_t s_count[RADIX];
    __shared__ uint32_t s_start[RADIX];
    __shared__ uint32_t s_delta[RADIX];
    __shared__ __attribute__((aligned(16))) KV<KeyT> s_kv[TILE];
    // SEG: the segment of each staged element, relative to the tile's first
    __shared__ uint8_t s_seg[SEG ? TILE : 1];
    __shared__ uint32_t s_bound[SEG ? kTileSegs : 1];
    // during ranking the start of s_kv holds one 64-bit lane mask per digit
    // per wave (it is staged into only afterwards)
    static_assert((size_t)WAVES * RADIX * 8 <= sizeof(KV<KeyT>) * TILE, "peer masks fit in s_kv");
    unsigned long long* s_mask = (unsigned long long*)s_kv;

    KeyT key[ITEMS];
    uint32_t idx[ITEMS], dig[ITEMS], rank[ITEMS];
    // With the default tile order the tile is known from the block index, so
    // (one list) its elements are loaded before the status and the schedule
    // are read, from the buffer `exp_in` the host expects when no pattern is
    // skipped (pairs of this kernel's width, or packed words); a pass whose
    // input is elsewhere loads again below.  The addresses are valid whatever
    // the buffers hold.
    bool early = false;
    if constexpr (!SEG && sizeof(Pair<KeyT>) == 8) {
        const bool packed_exp = buf_packed(exp_in);
        const bool pairs_exp = HI ? buf_half(exp_in) : buf_pairs(exp_in);
        if (!ticket && (packed_exp || pairs_exp)) {
            const uint32_t q0 = blockIdx.x / 8u;
            const uint64_t t0 = (uint64_t)((q0 / kPassChunk) * (8u * kPassChunk) +
                                           (blockIdx.x % 8u) * kPassChunk + q0 % kPassChunk);
            const uint64_t wb = t0 * TILE + (uint64_t)(threadIdx.x / 64) * (64 * ITEMS);
            const uint32_t ln = threadIdx.x % 64;
            const Pair<KeyT>* src = buf_in_b(exp_in) ? pairsB : pairsA;
            early = true;
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                const uint64_t e = wb + (uint64_t)i * 64 + ln;
                key[i] = 0;
                idx[i] = 0;
                if (e < n_all) {
                    if (packed_exp) {
                        idx[i] = ((const uint32_t*)src)[e];
                    } else {
                        const Pair<KeyT> v = src[e];
                        key[i] = pair_key<KeyT>(v);
                        idx[i] = v.idx;
                    }
                }
            }
        }
    }

    if (hdr->status != 0)
        return;
    const PassSched ps = hdr->sched[pass];
    if (ps.skip)
        return;
    // the number of elements: the whole list, or (SEG) the lists that take
    // the passes, known on the device only
    const uint32_t n = SEG ? hdr->seg_nodes : n_all;
    const uint32_t nseg = SEG ? hdr->n_segs : 0u;
    static_assert(!HI || (sizeof(KeyT) == 4 && !SEG), "high-half passes are 32-bit, one list");
    // this kernel's own pairs: Pair<KeyT>, or (HI) the half pairs
    const bool out_pairs = HI ? buf_half(ps.out_kind) : buf_pairs(ps.out_kind);
    const bool out_packed = buf_packed(ps.out_kind);
    // (64-bit keys) pairs over the high half for the passes that follow
    const bool out_half = !HI && sizeof(KeyT) == 8 && !SEG && buf_half(ps.out_kind);
    const bool in_packed = buf_packed(ps.in_kind);
    // (HI) the full 64-bit pairs, read for their high half
    const bool in_wide = HI && buf_pairs(ps.in_kind);
    const bool in_b = buf_in_b(ps.in_kind), out_b = buf_in_b(ps.out_kind);
    const Pair<KeyT>* pin = in_b ? pairsB : pairsA;
    Pair<KeyT>* pout = out_b ? pairsB : pairsA;
    uint32_t* iout = ps.out_kind == kBufIdxB ? idxB : idxA;
    // packed words: digit in the top RB bits, node index below
    constexpr uint32_t PK = 32u - RB;
    const uint32_t* uin = (const uint32_t*)pin;
    uint32_t* uout = (uint32_t*)pout;
    const Pair<uint64_t>* win = (const Pair<uint64_t>*)pin;
    Pair<uint32_t>* hout = (Pair<uint32_t>*)pout;

    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / 64, lane = tid % 64;
    __shared__ uint32_t s_tile;
    if (ticket && tid == 0)
        s_tile = atomicAdd(&hdr->pass_ticket[pass], 1u);
    for (uint32_t i = tid; i < WAVES * RADIX; i += BLOCK) {
        (&s_wave[0][0])[i] = 0;
        s_mask[i] = 0ull;
    }
    __syncthreads();
    const uint32_t q = blockIdx.x / 8u;
    const uint32_t tile = ticket ? s_tile
                                 : (q / kPassChunk) * (8u * kPassChunk) +
                                       (blockIdx.x % 8u) * kPassChunk + q % kPassChunk;
    if ((uint64_t)tile * TILE >= (uint64_t)n)
        return;  // the grid is rounded up to whole chunk groups (SEG: to all nodes)
    const uint64_t tbase = (uint64_t)tile * TILE;
    const uint64_t wbase = tbase + (uint64_t)wave * (64 * ITEMS);
    uint32_t seg0 = 0, nb = 0;
    if constexpr (SEG) {
        // the segments this tile spans: boundaries relative to its first one
        seg0 = seg_of(sm, (uint32_t)tbase, nseg);
        const uint32_t tend = (uint32_t)min<uint64_t>(tbase + TILE, (uint64_t)n);
        if (tid < kTileSegs) {
            const uint32_t sidx = seg0 + 1 + tid;
            s_bound[tid] = sidx < nseg ? sm.coff[sidx] : 0xFFFFFFFFu;
        }
        for (uint32_t k = 0; k < kTileSegs; k++)
            nb += (seg0 + 1 + k < nseg) && (sm.coff[seg0 + 1 + k] < tend);
        __syncthreads();
    }

    if (early && ps.in_kind == exp_in) {
        // the elements loaded early: digits (packed words: digit and node)
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint64_t e = wbase + (uint64_t)i * 64 + lane;
            if (e < n) {
                if (in_packed) {
                    const uint32_t v = idx[i];
                    dig[i] = v >> PK;
                    idx[i] = v & ((1u << PK) - 1u);
                    key[i] = (KeyT)((KeyT)dig[i] << shift);
                } else {
                    dig[i] = (uint32_t)(key[i] >> shift) & (RADIX - 1u);
                }
            } else {
                key[i] = 0;
                idx[i] = 0;
                dig[i] = RADIX;
            }
        }
    } else if (!SEG && in_packed) {
        // the key is only needed for this pass's digit: it is kept in place
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint64_t e = wbase + (uint64_t)i * 64 + lane;
            if (e < n) {
                const uint32_t v = uin[e];
                dig[i] = v >> PK;
                idx[i] = v & ((1u << PK) - 1u);
                key[i] = (KeyT)((KeyT)dig[i] << shift);
            } else {
                key[i] = 0;
                idx[i] = 0;
                dig[i] = RADIX;
            }
        }
    } else if (HI && in_wide) {
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint64_t e = wbase + (uint64_t)i * 64 + lane;
            if (e < n) {
                const Pair<uint64_t> v = win[e];
                key[i] = (KeyT)v.khi;
                idx[i] = v.idx;
                dig[i] = (uint32_t)(key[i] >> shift) & (RADIX - 1u);
            } else {
                key[i] = 0;
                idx[i] = 0;
                dig[i] = RADIX;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint64_t e = wbase + (uint64_t)i * 64 + lane;
            if (e < n) {
                const Pair<KeyT> v = pin[e];
                key[i] = pair_key<KeyT>(v);
                idx[i] = v.idx;
                dig[i] = (uint32_t)(key[i] >> shift) & (RADIX - 1u);
                if constexpr (SEG) {
                    uint32_t sl = 0;
                    while (sl < nb && s_bound[sl] <= (uint32_t)e)
                        sl++;
                    dig[i] |= sl << 9;
                }
            } else {
                key[i] = 0;
                idx[i] = 0;
                dig[i] = RADIX;
            }
        }
    }
    // dig[i] bits: 0..8 digit (RADIX = invalid), 9..15 segment slot (SEG),
    // 16..21 rank in the wave's group, 24..29 the group's first lane (which
    // holds the LDS base)
    const uint64_t lt = lanemask_lt();
    unsigned long long* w_mask = s_mask + (size_t)wave * RADIX;
    const bool by_ballot = ps.ballot != 0;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint32_t d = dig[i] & 0x1FFu;
        const bool valid = d < RADIX;
        // peers = the lanes of this wave whose item i has the same digit
        uint64_t peers;
        if (by_ballot) {
            // K ballots: a cost independent of the digit mix
            peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < RB; b++) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
        } else {
            // each lane ORs its bit into its digit's mask, reads the mask
            // back, and clears it.  OR is order-independent, so the mask is
            // exact however the LDS serialises lanes that hit the same word;
            // a wave's LDS operations complete in issue order.
            if (valid)
                __hip_atomic_fetch_or(&w_mask[d], 1ull << lane, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WAVEFRONT);
            __builtin_amdgcn_wave_barrier();
            peers = valid ? (uint64_t)__hip_atomic_load(&w_mask[d], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WAVEFRONT)
                          : 0ull;
            __builtin_amdgcn_wave_barrier();
            if (valid)
                __hip_atomic_store(&w_mask[d], 0ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
            __builtin_amdgcn_wave_barrier();
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t first = valid ? (uint32_t)(__ffsll((unsigned long long)peers) - 1) : lane;
        uint32_t base = 0;
        if (valid && below == 0)
            base = atomicAdd(&s_wave[wave][d], (uint32_t)__popcll(peers));
        rank[i] = base;
        dig[i] |= (below << 16) | (first << 24);
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        rank[i] = __shfl(rank[i], (int)(dig[i] >> 24), 64) + ((dig[i] >> 16) & 0xFFu);
        dig[i] &= 0xFFFFu;
    }
    __syncthreads();
    // per digit: exclusive offsets across waves and the tile count
    for (uint32_t d = tid; d < RADIX; d += BLOCK) {
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t w = 0; w < WAVES; w++) {
            const uint32_t v = s_wave[w][d];
            s_wave[w][d] = sum;
            sum += v;
        }
        s_count[d] = sum;
        // publish this tile's count early so successors can proceed
        st_agent(&look[(size_t)tile * RADIX + d], (tile == 0 ? LK::PREFIX : LK::AGG) | (LW)sum);
    }
    __syncthreads();
    // local digit starts (exclusive scan over digits) by wave 0
    if (wave == 0) {
        constexpr uint32_t PER = (RADIX + 63) / 64;
        uint32_t vals[PER];
        uint32_t local = 0;
#pragma unroll
        for (uint32_t j = 0; j < PER; j++) {
            const uint32_t d = lane * PER + j;
            vals[j] = d < RADIX ? s_count[d] : 0;
            local += vals[j];
        }
        uint32_t incl = local;
#pragma unroll
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t up = __shfl_up(incl, off, 64);
            if (lane >= off)
                incl += up;
        }
        uint32_t run = incl - local;
#pragma unroll
        for (uint32_t j = 0; j < PER; j++) {
            const uint32_t d = lane * PER + j;
            if (d < RADIX)
                s_start[d] = run;
            run += vals[j];
        }
    }
    __syncthreads();
    // each wave's offset within a digit becomes its offset within the tile,
    // so staging reads one table entry per item
    for (uint32_t i = tid; i < WAVES * RADIX; i += BLOCK)
        (&s_wave[0][0])[i] += s_start[i % RADIX];
    __syncthreads();
    // decoupled look-back per digit, kLookWindow predecessors per round trip:
    // the window's words are loaded together and consumed in tile order up to
    // the first inclusive prefix; an unpublished word stops the consumption
    // there (later words of the window are not used past it)
    for (uint32_t d = tid; d < RADIX; d += BLOCK) {
        uint32_t excl = 0;
        if (tile != 0) {
            int64_t j = (int64_t)tile - 1;  // the next predecessor to add
            uint32_t spins = 0;
            bool done = false;
            while (!done && j >= 0) {
                LW v[kLookWindow];
#pragma unroll
                for (uint32_t w = 0; w < kLookWindow; w++)
                    v[w] = (j >= (int64_t)w) ? ld_agent(&look[(size_t)(j - w) * RADIX + d]) : (LW)0;
                uint32_t used = 0;
                bool blocked = false;
#pragma unroll
                for (uint32_t w = 0; w < kLookWindow; w++) {
                    if (done || blocked || j < (int64_t)w)
                        continue;
                    const LW f = v[w] & ~LK::MASK;
                    if (f == 0) {
                        blocked = true;
                        continue;
                    }
                    excl += (uint32_t)(v[w] & LK::MASK);
                    used = w + 1;
                    if (f == LK::PREFIX)
                        done = true;
                }
                j -= used;
                if (done || used > 0) {
                    spins = 0;
                    continue;
                }
                // predecessor j has published nothing yet
                if (++spins <= spin_limit) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                // predecessor not running yet: count its digit d directly
                const uint64_t b0 = (uint64_t)j * TILE;
                const uint64_t b1 = min<uint64_t>(b0 + TILE, (uint64_t)n);
                uint32_t c = 0;
                if (!SEG && in_packed) {
                    for (uint64_t q = b0; q < b1; q++)
                        c += (uin[q] >> PK) == d;
                } else if (HI && in_wide) {
                    for (uint64_t q = b0; q < b1; q++)
                        c += ((win[q].khi >> shift) & (RADIX - 1u)) == d;
                } else {
                    for (uint64_t q = b0; q < b1; q++)
                        c += ((uint32_t)(pair_key<KeyT>(pin[q]) >> shift) & (RADIX - 1u)) == d;
                }
                excl += c;
                j--;
                spins = 0;
            }
            st_agent(&look[(size_t)tile * RADIX + d], LK::PREFIX | (LW)(excl + s_count[d]));
        }
        // wrapping u32 arithmetic: position = j + (base - local start), the
        // base of SEG lists added per element
        // (SEG: a tile inside one segment folds that segment's base in here;
        // otherwise each element adds its own segment's base below)
        const uint32_t base = SEG ? (nb == 0 ? sm.lbase[(size_t)seg0 * RADIX + d] : 0u) : dbase[d];
        s_delta[d] = base + excl - s_start[d];
    }
    // stage the tile in LDS grouped by digit (stable)
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint32_t d = dig[i] & 0x1FFu;
        if (d < RADIX) {
            const uint32_t pos = s_wave[wave][d] + rank[i];
            KV<KeyT> kv;
            kv.key = key[i];
            kv.idx = idx[i];
            s_kv[pos] = kv;
            if constexpr (SEG) {
                if (nb != 0)
                    s_seg[pos] = (uint8_t)(dig[i] >> 9);
            }
        }
    }
    __syncthreads();
    const uint32_t valid_n = (uint32_t)min<uint64_t>((uint64_t)TILE, (uint64_t)n - tbase);
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint32_t j = tid + i * BLOCK;
        if (j < valid_n) {
            const KV<KeyT> kv = s_kv[j];
            const uint32_t d = (uint32_t)(kv.key >> shift) & (RADIX - 1u);
            uint32_t g = j + s_delta[d];
            if constexpr (SEG) {
                if (nb != 0)
                    g += sm.lbase[(size_t)(seg0 + s_seg[j]) * RADIX + d];
            }
            if (g < n) {
                if (out_pairs)
                    pout[g] = make_pair_kv<KeyT>(kv.key, kv.idx);
                else if (out_half)
                    hout[g] = make_pair_kv<uint32_t>((uint32_t)((uint64_t)kv.key >> 32), kv.idx);
                else if (!SEG && out_packed)
                    uout[g] = (((uint32_t)(kv.key >> ps.pk_shift) & (RADIX - 1u)) << PK) | kv.idx;
                else
                    iout[g] = kv.idx;
            }
        }
    }
}

// ---------------------------------------------------------------- short lists
// One workgroup sorts one list of at most CUT nodes entirely in LDS:
//   1. its links (list-local) and keys are read once;
//   2. pointer jumping (Wyllie) gives every node its distance to the end; the
//      list is well formed iff, after ceil(log2 len) rounds, the head's
//      pointer is NIL and its distance is len (its path then visits all len
//      nodes); position = len - distance;
//   3. the (key, node) pairs are placed in list order and split stably on
//      every K-bit pattern, least significant first (ballot ranking per
//      wave, counts scanned across waves), in LDS;
//   4. the new links (list-local, NIL at the end) are built in LDS in index
//      order.
// Returns false for a malformed list (a link outside the list, or a head whose
// path does not visit every node), true otherwise with `links` pointing at the
// new links in LDS and `new_head` the list-local new head.  Called by every
// thread of a kSmallThreads workgroup; `head` is list-local and below len.
constexpr int kSmallThreads = 512;

template <typename KeyT, int RB, int CUT>
__device__ __forceinline__ bool small_sort(const uint32_t* __restrict__ nxt,
                                           const KeyT* __restrict__ kp, uint32_t len,
                                           uint32_t shift_in, uint32_t head, KeyT float_sel,
                                           KeyT xor_mask, uint32_t passes,
                                           const uint32_t*& links, uint32_t& new_head)
{
    constexpr int T = kSmallThreads;
    constexpr int IT = CUT / T;
    constexpr uint32_t WAVES = T / 64;
    constexpr uint32_t RADIX = 1u << RB;
    constexpr size_t RAW = sizeof(KV<KeyT>) > 8 ? sizeof(KV<KeyT>) : 8;
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[RAW * CUT];
    __shared__ uint32_t s_next[CUT];
    __shared__ uint32_t s_wave[WAVES][RADIX];
    __shared__ uint32_t s_start[RADIX];
    __shared__ int s_trivial;
    uint2* s_ps = (uint2*)s_raw;        // ranking: (pointer, distance)
    KV<KeyT>* s_kv = (KV<KeyT>*)s_raw;  // sorting: (key, node) in list order
    const uint32_t tid = threadIdx.x, wave = tid / 64, lane = tid % 64;

    uint32_t ptr[IT], dist[IT];
    KeyT key[IT];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < IT; k++) {
        const uint32_t i = tid + k * T;
        ptr[k] = kNil;
        dist[k] = 0;
        key[k] = 0;
        if (i < len) {
            uint32_t x = nxt[i];
            if (x != kNil) {
                x -= shift_in;  // wraps to >= len when outside the slab
                if (x >= len) {
                    bad = true;
                    x = kNil;
                }
            }
            ptr[k] = x;
            dist[k] = 1;
            key[k] = transform_key<KeyT>(kp[i], float_sel, xor_mask);
            s_ps[i] = make_uint2(x, 1u);
        }
    }
    __syncthreads();
    uint32_t rounds = 0;
    while ((1u << rounds) < len)
        rounds++;
    for (uint32_t r = 0; r < rounds; r++) {
#pragma unroll
        for (int k = 0; k < IT; k++) {
            if (ptr[k] != kNil) {
                const uint2 q = s_ps[ptr[k]];
                ptr[k] = q.x;
                dist[k] += q.y;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IT; k++) {
            const uint32_t i = tid + k * T;
            if (i < len)
                s_ps[i] = make_uint2(ptr[k], dist[k]);
        }
        __syncthreads();
    }
    const uint2 hq = s_ps[head];
    bad |= hq.x != kNil || hq.y != len;
    if (__syncthreads_or(bad))
        return false;
    // list order: the pair of node i goes to position len - dist
#pragma unroll
    for (int k = 0; k < IT; k++) {
        const uint32_t i = tid + k * T;
        if (i < len) {
            KV<KeyT> kv;
            kv.key = key[k];
            kv.idx = i;
            s_kv[len - dist[k]] = kv;
        }
    }
    for (uint32_t i = tid; i < WAVES * RADIX; i += T)
        (&s_wave[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    for (uint32_t p = 0; p < passes; p++) {
        const uint32_t shift = p * RB;
        KV<KeyT> kv[IT];
        uint32_t dig[IT], rank[IT];
#pragma unroll
        for (int k = 0; k < IT; k++) {
            const uint32_t e = wave * (64 * IT) + k * 64 + lane;
            if (e < len) {
                kv[k] = s_kv[e];
                dig[k] = (uint32_t)(kv[k].key >> shift) & (RADIX - 1u);
            } else {
                kv[k].key = 0;
                kv[k].idx = 0;
                dig[k] = RADIX;
            }
        }
        // ballot ranking in wave order, items in program order
#pragma unroll
        for (int k = 0; k < IT; k++) {
            const bool valid = dig[k] < RADIX;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < RB; b++) {
                const bool bit = (dig[k] >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const uint32_t below = (uint32_t)__popcll(peers & lt);
            const uint32_t first = valid ? (uint32_t)(__ffsll((unsigned long long)peers) - 1) : lane;
            uint32_t base = 0;
            if (valid && below == 0)
                base = atomicAdd(&s_wave[wave][dig[k]], (uint32_t)__popcll(peers));
            rank[k] = __shfl(base, (int)first, 64) + below;
        }
        if (tid == 0)
            s_trivial = 0;
        __syncthreads();
        for (uint32_t d = tid; d < RADIX; d += T) {
            uint32_t sum = 0;
#pragma unroll
            for (uint32_t w = 0; w < WAVES; w++) {
                const uint32_t v = s_wave[w][d];
                s_wave[w][d] = sum;
                sum += v;
            }
            s_start[d] = sum;
            if (sum == len)
                s_trivial = 1;  // every node has digit d: the pass is the identity
        }
        __syncthreads();
        if (wave == 0) {
            constexpr uint32_t PER = (RADIX + 63) / 64;
            uint32_t vals[PER];
            uint32_t local = 0;
#pragma unroll
            for (uint32_t j = 0; j < PER; j++) {
                const uint32_t d = lane * PER + j;
                vals[j] = d < RADIX ? s_start[d] : 0;
                local += vals[j];
            }
            uint32_t incl = local;
#pragma unroll
            for (uint32_t off = 1; off < 64; off <<= 1) {
                const uint32_t up = __shfl_up(incl, off, 64);
                if (lane >= off)
                    incl += up;
            }
            uint32_t run = incl - local;
#pragma unroll
            for (uint32_t j = 0; j < PER; j++) {
                const uint32_t d = lane * PER + j;
                if (d < RADIX)
                    s_start[d] = run;
                run += vals[j];
            }
        }
        __syncthreads();
        if (!s_trivial) {
#pragma unroll
            for (int k = 0; k < IT; k++)
                if (dig[k] < RADIX)
                    s_kv[s_start[dig[k]] + s_wave[wave][dig[k]] + rank[k]] = kv[k];
        }
        __syncthreads();
        for (uint32_t i = tid; i < WAVES * RADIX; i += T)
            (&s_wave[0][0])[i] = 0;
        __syncthreads();
    }
    // new links in LDS, then out in index order
    for (uint32_t j = tid; j < len; j += T)
        s_next[s_kv[j].idx] = (j + 1 < len) ? s_kv[j + 1].idx : kNil;
    new_head = s_kv[0].idx;
    __syncthreads();
    links = s_next;
    return true;
}


}  // namespace pbit
