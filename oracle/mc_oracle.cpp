// Plain CPU oracle for the minhash metagenomic classifier of
// "MetaCache-GPU: Ultra-Fast Metagenomic Classification" (Kobus et al., ICPP'21).
//
// TEST INFRASTRUCTURE ONLY. This file is the checker: only the tests, the smoke
// check and the CPU-baseline leg of the benchmark load it. It shares no code,
// header, table or constant with the HIP library and never calls it.
//
// It computes the definitions of the method directly and slowly: one k-mer at a
// time, std::set for sketches, std::multimap for the index, per-read brute-force
// scoring, and LCA by walking parent links. Readings taken where the paper is
// silent are marked "Reading:" below.
//
// Location encoding (shared by both sides only as an output format):
//   location = (target << 18) | window, target < 2^14 - 1, window < 2^18.
//
// Parity status per function:
//   h1 (fmix32)            pinned: published MurmurHash3 vectors + inverse.
//   kmers / canonical      pinned: brute-force string enumeration.
//   bottom_s / sketches    pinned: the paper's worked minhash example (Sec. 2),
//                          reverse-complement invariance, set semantics.
//   windows                pinned: closed form ceil((L-k+1)/S), partition.
//   index + cap            pinned: two cap strategies agree, pair counts,
//                          repeated-genome stress outcome, incremental build.
//   scoring / top / label  pinned: brute force over every (target, start).
//   lca                    pinned: hand-worked cases, ancestor-set brute force.
//   h1 vs the paper        parity unpinned: the paper does not define h1.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <thread>
#include <unordered_set>
#include <vector>

namespace {

const uint32_t kUnclassified = 0xFFFFFFFFu;
const uint32_t kWindowBits = 18;
const uint32_t kMaxTargets = (1u << 14) - 1;      // ids 0 .. 16382
const uint32_t kMaxWindows = 1u << kWindowBits;

// Sec. 5.2 (step 1) and Sec. 5.3: nucleotides A, C, G, T are coded in two bits;
// ambiguous characters are tracked separately and no valid k-mer may cover one.
// Reading: lower-case letters are the same bases; every other byte is invalid.
int base_code(unsigned char c) {
    switch (c) {
        case 'A': case 'a': return 0;
        case 'C': case 'c': return 1;
        case 'G': case 'g': return 2;
        case 'T': case 't': return 3;
        default: return -1;
    }
}

// h1 (Sec. 4.1). The paper leaves h1 open. Reading: the 32-bit finalizer of
// MurmurHash3 (Appleby, public domain), a bijection on 32-bit words.
uint32_t h1(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// Canonical k-mer (Sec. 4.1) at position pos. The forward value reads the k
// bases with the first base most significant; the reverse complement reads the
// bases backwards with each base complemented (3 - code). The canonical value
// is the smaller of the two. Returns false if a base is not A/C/G/T.
bool canonical_kmer(const unsigned char* seq, uint64_t pos, uint32_t k, uint32_t* out) {
    uint64_t fwd = 0, rev = 0;
    for (uint32_t i = 0; i < k; ++i) {
        int c = base_code(seq[pos + i]);
        if (c < 0) return false;
        fwd = fwd * 4 + (uint64_t)c;
    }
    for (uint32_t i = 0; i < k; ++i) {
        int c = base_code(seq[pos + k - 1 - i]);
        rev = rev * 4 + (uint64_t)(3 - c);
    }
    *out = (uint32_t)std::min(fwd, rev);
    return true;
}

// Windows (Sec. 4.1, Sec. 5.2): windows of w bases overlap by k-1, so their
// starts are S = w-k+1 apart and every k-mer start belongs to exactly one window.
// Reading: a sequence of length L >= k has ceil((L-k+1)/S) windows, the last one
// possibly shorter; a sequence shorter than k has none.
uint64_t num_windows(uint64_t len, uint32_t k, uint32_t w) {
    if (len < k) return 0;
    uint64_t S = w - k + 1;
    uint64_t starts = len - k + 1;
    return (starts + S - 1) / S;
}

// Minhash sketch (Sec. 2, Sec. 5.3): the s smallest distinct hash values, in
// ascending order. Fewer than s distinct values give a shorter sketch.
std::vector<uint32_t> bottom_s(const std::vector<uint32_t>& values, uint32_t s) {
    std::set<uint32_t> distinct(values.begin(), values.end());
    std::vector<uint32_t> out;
    for (uint32_t v : distinct) {
        if (out.size() == s) break;
        out.push_back(v);
    }
    return out;
}

// Sketch of window j of a sequence: h1 of every valid canonical k-mer whose
// start lies in [jS, min((j+1)S, L-k+1)), then the bottom-s selection.
std::vector<uint32_t> window_sketch(const unsigned char* seq, uint64_t len, uint32_t k,
                                    uint32_t w, uint32_t s, uint64_t j) {
    uint64_t S = w - k + 1;
    uint64_t first = j * S;
    uint64_t last = std::min((j + 1) * S, len - k + 1);
    std::vector<uint32_t> hashes;
    for (uint64_t p = first; p < last; ++p) {
        uint32_t canon;
        if (canonical_kmer(seq, p, k, &canon)) hashes.push_back(h1(canon));
    }
    return bottom_s(hashes, s);
}

// sws (Sec. 5.6): the largest number of reference windows a fragment of length
// F can touch with its k-mers. Reading: ceil((F-k)/S) + 1 for F >= k, else 1.
uint32_t sliding_window_size(uint64_t F, uint32_t k, uint32_t w) {
    if (F < k) return 1;
    uint64_t S = w - k + 1;
    return (uint32_t)((F - k + S - 1) / S + 1);
}

struct Db {
    uint32_t k, w, s, cap;
    std::multimap<uint32_t, uint32_t> index;      // feature -> location
    std::vector<uint32_t> target_taxon;
    std::vector<uint32_t> parents;
    std::unordered_set<uint32_t> filter;          // features kept when filtering
    bool use_filter = false;
    uint32_t range_lo = 1, range_hi = 0;          // also kept: lo <= feature <= hi
};

// Cap (Sec. 4.1): at most `cap` locations per feature. The CPU index appends
// locations in ascending (target, window) order and stops at the cap, so the
// survivors are the `cap` smallest locations. Reading: keep exactly those.
void apply_cap(Db* db) {
    auto& idx = db->index;
    for (auto it = idx.begin(); it != idx.end();) {
        auto range = idx.equal_range(it->first);
        size_t n = (size_t)std::distance(range.first, range.second);
        if (n > db->cap) {
            std::vector<uint32_t> locs;
            for (auto e = range.first; e != range.second; ++e) locs.push_back(e->second);
            std::sort(locs.begin(), locs.end());
            uint32_t limit = locs[db->cap - 1];
            for (auto e = range.first; e != range.second;) {
                if (e->second > limit) e = idx.erase(e);
                else ++e;
            }
        }
        it = idx.upper_bound(it->first);
    }
}

// All (feature, location) pairs of one target, in ascending window order.
void target_pairs(const Db* db, const unsigned char* seq, uint64_t len, uint32_t target,
                  std::vector<std::pair<uint32_t, uint32_t>>* out) {
    uint64_t nw = num_windows(len, db->k, db->w);
    for (uint64_t j = 0; j < nw; ++j) {
        for (uint32_t f : window_sketch(seq, len, db->k, db->w, db->s, j)) {
            if (db->use_filter && !db->filter.count(f) &&
                !(f >= db->range_lo && f <= db->range_hi))
                continue;
            out->push_back({f, (target << kWindowBits) | (uint32_t)j});
        }
    }
}

int check_targets(const Db* db, const uint64_t* lengths, uint32_t n) {
    if ((uint64_t)db->target_taxon.size() + n > kMaxTargets) return -2;
    for (uint32_t i = 0; i < n; ++i)
        if (num_windows(lengths[i], db->k, db->w) > kMaxWindows) return -2;
    return 0;
}

// Build (Sec. 4.1): every window's sketch element is inserted with its location.
int add_targets(Db* db, const unsigned char* genomes, const uint64_t* lengths,
                const uint32_t* taxa, uint32_t n, int n_threads) {
    int rc = check_targets(db, lengths, n);
    if (rc) return rc;
    std::vector<uint64_t> off(n + 1, 0);
    for (uint32_t i = 0; i < n; ++i) off[i + 1] = off[i] + lengths[i];
    uint32_t base = (uint32_t)db->target_taxon.size();
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> pairs(n);
    // Threads only split the targets; each target's pairs are computed by the
    // same plain code and inserted below in ascending target order.
    int T = std::max(1, n_threads);
    std::vector<std::thread> pool;
    for (int t = 0; t < T; ++t) {
        pool.emplace_back([&, t]() {
            for (uint32_t i = (uint32_t)t; i < n; i += (uint32_t)T)
                target_pairs(db, genomes + off[i], lengths[i], base + i, &pairs[i]);
        });
    }
    for (auto& th : pool) th.join();
    for (uint32_t i = 0; i < n; ++i) {
        for (auto& p : pairs[i]) db->index.insert(p);
        db->target_taxon.push_back(taxa[i]);
    }
    apply_cap(db);
    return 0;
}

// Second cap strategy, used only to pin the first: insert in ascending
// (target, window) order and skip a pair once its feature holds `cap` locations.
int add_targets_stop_at_cap(Db* db, const unsigned char* genomes, const uint64_t* lengths,
                            const uint32_t* taxa, uint32_t n) {
    int rc = check_targets(db, lengths, n);
    if (rc) return rc;
    uint64_t o = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t t = (uint32_t)db->target_taxon.size();
        std::vector<std::pair<uint32_t, uint32_t>> pairs;
        target_pairs(db, genomes + o, lengths[i], t, &pairs);
        for (auto& p : pairs)
            if (db->index.count(p.first) < db->cap) db->index.insert(p);
        db->target_taxon.push_back(taxa[i]);
        o += lengths[i];
    }
    return 0;
}

uint32_t depth_of(const Db* db, uint32_t x) {
    uint32_t d = 0;
    while (db->parents[x] != x) { x = db->parents[x]; ++d; }
    return d;
}

// Lowest common ancestor (Sec. 4.2): the deepest node that is an ancestor (or
// the node itself) of both a and b, found by lifting the deeper node and then
// walking both up together.
uint32_t lca(const Db* db, uint32_t a, uint32_t b) {
    uint32_t da = depth_of(db, a), db_ = depth_of(db, b);
    while (da > db_) { a = db->parents[a]; --da; }
    while (db_ > da) { b = db->parents[b]; --db_; }
    while (a != b) { a = db->parents[a]; b = db->parents[b]; }
    return a;
}

struct Hit { uint32_t target, score, window_begin; };

// Label rule (Sec. 4.2, Sec. 6.5): no candidate or a top score under the hit
// threshold leaves the read unclassified; a lead of more than hit_diff over the
// second score gives the top target's taxon; otherwise the LCA of the taxa of
// all listed targets whose score is within hit_diff of the top score.
uint32_t decide(const Db* db, const std::vector<Hit>& top, uint32_t min_hits, uint32_t hit_diff) {
    if (top.empty() || top[0].score < min_hits) return kUnclassified;
    uint32_t c1 = top[0].score;
    uint32_t c2 = top.size() > 1 ? top[1].score : 0;
    if (c1 - c2 > hit_diff) return db->target_taxon[top[0].target];
    uint32_t label = db->target_taxon[top[0].target];
    for (size_t i = 1; i < top.size(); ++i)
        if ((uint64_t)top[i].score + hit_diff >= c1)
            label = lca(db, label, db->target_taxon[top[i].target]);
    return label;
}

struct QueryOpts { uint32_t top_m, min_hits, hit_diff, insert_size, paired; };

// Query of one record (Sec. 4.2): every window of every mate is sketched as in
// the build; all sketch elements together (no de-duplication across windows)
// look up their location lists; equal locations are counted (window count
// statistic); for every target the best sum over `sws` consecutive windows is
// taken; targets are ranked by (score desc, target asc) and the first top_m kept.
// Reading: one candidate per target; its window_begin is the smallest hit window
// that starts a best range.
void classify_record(const Db* db, const unsigned char* m1, uint64_t l1,
                     const unsigned char* m2, uint64_t l2, const QueryOpts& o,
                     uint32_t* label, Hit* top_out) {
    std::vector<uint32_t> query;
    const unsigned char* segs[2] = {m1, m2};
    uint64_t lens[2] = {l1, l2};
    for (int g = 0; g < 2; ++g) {
        uint64_t nw = num_windows(lens[g], db->k, db->w);
        for (uint64_t j = 0; j < nw; ++j)
            for (uint32_t f : window_sketch(segs[g], lens[g], db->k, db->w, db->s, j))
                query.push_back(f);
    }
    // Reading: a record with two non-empty mates is a pair whose fragment
    // length is max(l1 + l2, insert_size); otherwise its length is l1 + l2.
    uint64_t F = l1 + l2;
    if (l1 > 0 && l2 > 0 && o.insert_size > F) F = o.insert_size;
    uint32_t sws = sliding_window_size(F, db->k, db->w);

    std::map<uint32_t, uint32_t> hits;      // location -> count
    for (uint32_t f : query) {
        auto range = db->index.equal_range(f);
        for (auto e = range.first; e != range.second; ++e) hits[e->second] += 1;
    }
    std::map<uint32_t, Hit> best;            // target -> best range
    for (auto& h : hits) {
        uint32_t t = h.first >> kWindowBits, w0 = h.first & (kMaxWindows - 1);
        uint32_t score = 0;
        for (uint32_t w = w0; w < w0 + sws; ++w) {
            auto it = hits.find((t << kWindowBits) | w);
            if (w < kMaxWindows && it != hits.end()) score += it->second;
        }
        auto b = best.find(t);
        if (b == best.end() || score > b->second.score) best[t] = Hit{t, score, w0};
    }
    std::vector<Hit> cand;
    for (auto& b : best) cand.push_back(b.second);
    std::sort(cand.begin(), cand.end(), [](const Hit& a, const Hit& b) {
        return a.score != b.score ? a.score > b.score : a.target < b.target;
    });
    if (cand.size() > o.top_m) cand.resize(o.top_m);
    *label = decide(db, cand, o.min_hits, o.hit_diff);
    if (top_out) {
        for (uint32_t i = 0; i < o.top_m; ++i)
            top_out[i] = i < cand.size() ? cand[i] : Hit{kUnclassified, 0, 0};
    }
}

}  // namespace

extern "C" {

uint32_t orc_h1(uint32_t x) { return h1(x); }

uint64_t orc_num_windows(uint64_t len, uint32_t k, uint32_t w) { return num_windows(len, k, w); }

uint32_t orc_sws(uint64_t F, uint32_t k, uint32_t w) { return sliding_window_size(F, k, w); }

// Canonical k-mers at every start 0 .. len-k; valid[p] = 0 where a base is invalid.
void orc_kmers(const unsigned char* seq, uint64_t len, uint32_t k, uint32_t* canon,
               uint8_t* valid) {
    if (len < k) return;
    for (uint64_t p = 0; p + k <= len; ++p) {
        uint32_t c = 0;
        valid[p] = canonical_kmer(seq, p, k, &c) ? 1 : 0;
        canon[p] = c;
    }
}

uint32_t orc_bottom_s(const uint32_t* values, uint32_t n, uint32_t s, uint32_t* out) {
    std::vector<uint32_t> v(values, values + n);
    std::vector<uint32_t> r = bottom_s(v, s);
    std::copy(r.begin(), r.end(), out);
    return (uint32_t)r.size();
}

// Sketches of all windows of one sequence: counts[j] and feats[j*s ..].
uint64_t orc_sketch_windows(const unsigned char* seq, uint64_t len, uint32_t k, uint32_t w,
                            uint32_t s, uint32_t* counts, uint32_t* feats) {
    uint64_t nw = num_windows(len, k, w);
    for (uint64_t j = 0; j < nw; ++j) {
        std::vector<uint32_t> sk = window_sketch(seq, len, k, w, s, j);
        counts[j] = (uint32_t)sk.size();
        for (size_t i = 0; i < sk.size(); ++i) feats[j * s + i] = sk[i];
    }
    return nw;
}

void* orc_db_create(uint32_t k, uint32_t w, uint32_t s, uint32_t cap) {
    if (k < 1 || k > 16 || w < k || s < 1 || cap < 1) return nullptr;
    Db* db = new Db();
    db->k = k; db->w = w; db->s = s; db->cap = cap;
    return db;
}

void orc_db_destroy(void* db) { delete static_cast<Db*>(db); }

// Restrict the index to the given features (used to classify a read sample
// exactly without holding the whole index: pairs of other features can never
// be looked up by that sample).
void orc_db_set_filter(void* h, const uint32_t* feats, uint64_t n) {
    Db* db = static_cast<Db*>(h);
    db->filter.clear();
    db->filter.insert(feats, feats + n);
    db->use_filter = true;
}

// Additionally keep every feature in [lo, hi] while filtering.
void orc_db_set_filter_range(void* h, uint32_t lo, uint32_t hi) {
    Db* db = static_cast<Db*>(h);
    db->range_lo = lo;
    db->range_hi = hi;
    db->use_filter = true;
}

int orc_db_add_targets(void* h, const unsigned char* genomes, const uint64_t* lengths,
                       const uint32_t* taxa, uint32_t n, int n_threads) {
    return add_targets(static_cast<Db*>(h), genomes, lengths, taxa, n, n_threads);
}

int orc_db_add_targets_stop_at_cap(void* h, const unsigned char* genomes,
                                   const uint64_t* lengths, const uint32_t* taxa, uint32_t n) {
    return add_targets_stop_at_cap(static_cast<Db*>(h), genomes, lengths, taxa, n);
}

void orc_db_set_taxonomy(void* h, const uint32_t* parents, uint32_t n) {
    Db* db = static_cast<Db*>(h);
    db->parents.assign(parents, parents + n);
}

uint64_t orc_db_num_pairs(void* h) { return static_cast<Db*>(h)->index.size(); }

uint64_t orc_db_num_features(void* h) {
    Db* db = static_cast<Db*>(h);
    uint64_t n = 0;
    for (auto it = db->index.begin(); it != db->index.end(); it = db->index.upper_bound(it->first))
        ++n;
    return n;
}

// Index as (feature, location) pairs sorted by feature, then location.
void orc_db_dump(void* h, uint32_t* feats, uint32_t* locs) {
    Db* db = static_cast<Db*>(h);
    std::vector<std::pair<uint32_t, uint32_t>> all(db->index.begin(), db->index.end());
    std::sort(all.begin(), all.end());
    for (size_t i = 0; i < all.size(); ++i) { feats[i] = all[i].first; locs[i] = all[i].second; }
}

uint32_t orc_lca(void* h, uint32_t a, uint32_t b) { return lca(static_cast<Db*>(h), a, b); }

// Label for a given ranked top list (targets/scores of length n).
uint32_t orc_decide(void* h, const uint32_t* targets, const uint32_t* scores, uint32_t n,
                    uint32_t min_hits, uint32_t hit_diff) {
    std::vector<Hit> top;
    for (uint32_t i = 0; i < n; ++i) top.push_back(Hit{targets[i], scores[i], 0});
    return decide(static_cast<Db*>(h), top, min_hits, hit_diff);
}

// Classify records [first, first+count). Single-end: offsets has n+1 entries;
// paired: 2n+1 entries (mate 1, mate 2 per record). out_top holds top_m
// {target, score, window_begin} triples per record (may be null).
int orc_classify(void* h, const unsigned char* reads, const uint64_t* offsets, uint64_t first,
                 uint64_t count, uint32_t top_m, uint32_t min_hits, uint32_t hit_diff,
                 uint32_t insert_size, uint32_t paired, uint32_t* out_labels, uint32_t* out_top,
                 int n_threads) {
    Db* db = static_cast<Db*>(h);
    if (top_m < 1) return -1;
    QueryOpts o{top_m, min_hits, hit_diff, insert_size, paired};
    int T = std::max(1, n_threads);
    std::vector<std::thread> pool;
    for (int t = 0; t < T; ++t) {
        pool.emplace_back([&, t]() {
            for (uint64_t r = first + (uint64_t)t; r < first + count; r += (uint64_t)T) {
                uint64_t a, b, c;
                if (paired) { a = offsets[2 * r]; b = offsets[2 * r + 1]; c = offsets[2 * r + 2]; }
                else { a = offsets[r]; b = offsets[r + 1]; c = b; }
                Hit* top = out_top ? reinterpret_cast<Hit*>(out_top) + (r - first) * top_m : nullptr;
                classify_record(db, reads + a, b - a, reads + b, c - b, o,
                                &out_labels[r - first], top);
            }
        });
    }
    for (auto& th : pool) th.join();
    return 0;
}

// Query features of records [first, first+count): all window sketch elements
// of all mates, concatenated (used to build a feature filter for a sample).
uint64_t orc_query_features(uint32_t k, uint32_t w, uint32_t s, const unsigned char* reads,
                            const uint64_t* offsets, uint64_t first, uint64_t count,
                            uint32_t paired, uint32_t* out, uint64_t out_cap) {
    uint64_t n = 0;
    for (uint64_t r = first; r < first + count; ++r) {
        uint64_t bounds[3];
        int nseg;
        if (paired) { bounds[0] = offsets[2 * r]; bounds[1] = offsets[2 * r + 1]; bounds[2] = offsets[2 * r + 2]; nseg = 2; }
        else { bounds[0] = offsets[r]; bounds[1] = offsets[r + 1]; nseg = 1; }
        for (int g = 0; g < nseg; ++g) {
            uint64_t len = bounds[g + 1] - bounds[g];
            uint64_t nw = num_windows(len, k, w);
            for (uint64_t j = 0; j < nw; ++j)
                for (uint32_t f : window_sketch(reads + bounds[g], len, k, w, s, j)) {
                    if (n < out_cap) out[n] = f;
                    ++n;
                }
        }
    }
    return n;
}

}  // extern "C"
