// BPE vocabulary tables on the device: the ranked merge list, a pair -> rank
// hash, and per-id expansions for decode. (The merge-round kernel is added
// alongside.)
#include <vector>

#include "common.hpp"

namespace dnatok {

static uint32_t mix_pair(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 13;
    return h;
}

int build_bpe_tables(dnatok_vocab *v) {
    BpeTables &t = v->bpe;
    const int32_t R = (int32_t)(v->h_merges.size() / 2);
    t.n_merges = R;
    const int32_t V = 10 + R;
    // expansions (uppercase bases) per id
    std::vector<int32_t> len(V, 1);
    std::vector<int64_t> off(V, 0);
    for (int id = 0; id < 5; ++id) len[id] = 0;
    int64_t total = 0;
    for (int32_t r = 0; r < R; ++r) {
        int64_t L = (int64_t)len[v->h_merges[2 * r]] + len[v->h_merges[2 * r + 1]];
        if (L > (1 << 20)) return set_error(DNATOK_EVOCAB, "merge %d expands to more than 2^20 bases", r);
        len[10 + r] = (int32_t)L;
    }
    int32_t mx = 1;
    for (int32_t id = 0; id < V; ++id) {
        off[id] = total;
        total += len[id];
        if (len[id] > mx) mx = len[id];
    }
    std::vector<uint8_t> chars((size_t)(total > 0 ? total : 1));
    const char *B = "ACGTN";
    for (int32_t id = 5; id <= 9; ++id) chars[off[id]] = (uint8_t)B[id - 5];
    for (int32_t r = 0; r < R; ++r) {
        int32_t a = v->h_merges[2 * r], b = v->h_merges[2 * r + 1], id = 10 + r;
        std::copy(chars.begin() + off[a], chars.begin() + off[a] + len[a], chars.begin() + off[id]);
        std::copy(chars.begin() + off[b], chars.begin() + off[b] + len[b], chars.begin() + off[id] + len[a]);
    }
    v->max_token_bytes = mx;

    // pair -> rank hash: slot holds ((left << 32) | right) + 1 (0 = empty) and,
    // in a parallel array, the rank; linear probing, load factor <= 1/2.
    uint32_t slots = 16;
    while (slots < 2u * (uint32_t)(R > 0 ? R : 1)) slots <<= 1;
    std::vector<uint64_t> keys(slots, 0);
    std::vector<int32_t> ranks(slots, -1);
    for (int32_t r = 0; r < R; ++r) {
        uint32_t a = (uint32_t)v->h_merges[2 * r], b = (uint32_t)v->h_merges[2 * r + 1];
        uint64_t key = (((uint64_t)a << 32) | b) + 1;
        uint32_t s = mix_pair(a, b) & (slots - 1);
        while (keys[s]) s = (s + 1) & (slots - 1);
        keys[s] = key;
        ranks[s] = r;
    }
    t.hash_mask = slots - 1;

    void *p = nullptr;
    DNATOK_HIP(hipMalloc(&p, sizeof(uint64_t) * slots + sizeof(int32_t) * slots));
    t.d_hash = static_cast<uint64_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_hash, keys.data(), sizeof(uint64_t) * slots, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMemcpy(reinterpret_cast<int32_t *>(t.d_hash + slots), ranks.data(), sizeof(int32_t) * slots,
                         hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, sizeof(int32_t) * 2 * (size_t)(R > 0 ? R : 1)));
    t.d_merges = static_cast<int32_t *>(p);
    if (R > 0)
        DNATOK_HIP(hipMemcpy(t.d_merges, v->h_merges.data(), sizeof(int32_t) * 2 * (size_t)R, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, sizeof(int32_t) * (size_t)V));
    t.d_tok_len = static_cast<int32_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_len, len.data(), sizeof(int32_t) * (size_t)V, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, sizeof(int64_t) * (size_t)V));
    t.d_tok_off = static_cast<int64_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_off, off.data(), sizeof(int64_t) * (size_t)V, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, chars.size()));
    t.d_tok_chars = static_cast<uint8_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_chars, chars.data(), chars.size(), hipMemcpyHostToDevice));
    return DNATOK_OK;
}

void free_bpe_tables(dnatok_vocab *v) {
    BpeTables &t = v->bpe;
    if (t.d_hash) (void)hipFree(t.d_hash);
    if (t.d_merges) (void)hipFree(t.d_merges);
    if (t.d_tok_len) (void)hipFree(t.d_tok_len);
    if (t.d_tok_off) (void)hipFree(t.d_tok_off);
    if (t.d_tok_chars) (void)hipFree(t.d_tok_chars);
    t = BpeTables();
}

}  // namespace dnatok
