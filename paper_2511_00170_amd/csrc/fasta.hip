// FASTA input into the 2-bit store and AHv2-format FASTA output (host code).
//
// Ingest (Implementations: FASTA is turned into 2-bit batches of headers,
// lengths and bases; Discussion: headers kept apart from the bases) reads
// every file once.  The record table (identifiers, source files, lengths,
// first blocks) stays on the host; the bases, with header lines and white
// space removed, go through two pinned staging buffers: while the GPU copies
// one chunk and packs it (ah_pack_pieces), the host fills the other.  A
// sequence that does not fit in the rest of a chunk is cut on a 64-base
// boundary of the sequence, so every piece starts on a store block.
//
// Many files (one genome per file is the usual case) are read by several
// host threads: each file is indexed in parallel, the store layout is fixed
// in file order, and the files are packed in parallel, each worker with its
// own staging buffers (pieces carry absolute store blocks, so the order in
// which they land does not matter).
//
// Output follows Supplementary, "Headers and outputs".
#include <errno.h>
#include <fcntl.h>
#include <stdio.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <atomic>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "ah.h"
#include "ah_internal.h"

#include "fasta_table.h"

namespace {

constexpr uint64_t kReadBytes = 16ull << 20;

// ASCII white space: space, tab, LF, VT, FF, CR.
struct SpaceTable {
    bool t[256];
    SpaceTable() {
        for (int i = 0; i < 256; i++) t[i] = false;
        t[' '] = t['\t'] = t['\n'] = t['\v'] = t['\f'] = t['\r'] = true;
    }
};
const SpaceTable kSpace;

// Does any byte of x lie below 0x21 (the white space bytes all do)?
inline bool any_below_0x21(uint64_t x) {
    return ((x - 0x2121212121212121ull) & ~x & 0x8080808080808080ull) != 0;
}

// Copy src[0:n) to dst without white space; returns the bytes kept.  dst must
// hold n bytes.
inline size_t copy_bases(uint8_t *dst, const uint8_t *src, size_t n) {
    size_t k = 0, i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t x;
        memcpy(&x, src + i, 8);
        if (!any_below_0x21(x)) {
            memcpy(dst + k, &x, 8);
            k += 8;
            continue;
        }
        for (int j = 0; j < 8; j++) {
            const uint8_t c = src[i + j];
            dst[k] = c;
            k += !kSpace.t[c];
        }
    }
    for (; i < n; i++) {
        const uint8_t c = src[i];
        dst[k] = c;
        k += !kSpace.t[c];
    }
    return k;
}

inline size_t count_bases(const uint8_t *src, size_t n) {
    size_t k = 0, i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t x;
        memcpy(&x, src + i, 8);
        if (!any_below_0x21(x)) {
            k += 8;
            continue;
        }
        for (int j = 0; j < 8; j++) k += !kSpace.t[src[i + j]];
    }
    for (; i < n; i++) k += !kSpace.t[src[i]];
    return k;
}

inline uint64_t pieces_per_chunk(uint64_t chunk) { return chunk / 64 + 16; }

struct Slot {
    uint8_t *h_buf = nullptr;
    ah_pack_piece *h_pcs = nullptr;
    uint8_t *d_buf = nullptr;
    ah_pack_piece *d_pcs = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    uint64_t nbytes = 0;
    uint32_t npcs = 0;
};

struct Ingest {
    ah_fasta *f = nullptr;
    bool device = false;
    uint64_t chunk = 0;
    uint32_t pcap = 0;
    Slot slot[2];
    int cur = 0;
    hipStream_t s = nullptr;
    uint32_t *d_blocks = nullptr;
    uint64_t blocks_cap = 0;
    uint32_t *d_nbits = nullptr;
    uint64_t *d_counters = nullptr;
    uint64_t *d_nlist = nullptr;
    uint64_t nlist_cap = 0;
    ah_status err = AH_OK;
    // current record
    bool in_rec = false;
    uint64_t rec_len = 0;
    uint64_t rec_block0 = 0;
    int64_t piece = -1;  // the record's open piece in slot[cur], always its last

    void fail(ah_status e) {
        if (!err) err = e;
    }

    void begin_record(uint32_t fi) {
        if (f->len.size() >= 0xFFFFFFFFull) fail(AH_E_FORMAT);
        f->id_off.push_back(f->ids.size());
        f->file.push_back(fi);
        in_rec = true;
        rec_len = 0;
        rec_block0 = f->n_blocks;
        piece = -1;
    }

    void end_record() {
        f->ids.push_back('\0');
        if (rec_len >= (1ull << 32)) fail(AH_E_FORMAT);
        const uint32_t L = (uint32_t)rec_len;
        f->len.push_back(L);
        f->block0.push_back(rec_block0);
        f->n_blocks += (rec_len + 63) / 64;
        f->n_bases += rec_len;
        if (L > f->max_len) f->max_len = L;
        if (piece >= 0 && slot[cur].h_pcs[piece].n == 0) slot[cur].npcs--;
        piece = -1;
        in_rec = false;
    }

    void submit(int i) {
        Slot &S = slot[i];
        if (!S.npcs || err) return;
        if (hipMemcpyAsync(S.d_buf, S.h_buf, S.nbytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(S.d_pcs, S.h_pcs, S.npcs * sizeof(ah_pack_piece), hipMemcpyHostToDevice, s) !=
                hipSuccess) {
            fail(AH_E_HIP);
            return;
        }
        ah_status e = ah_pack_pieces(d_blocks, blocks_cap, d_nbits, d_counters, S.d_buf, S.d_pcs, S.npcs, d_nlist,
                                     nlist_cap, s);
        if (e) {
            fail(e);
            return;
        }
        if (hipEventRecord(S.ev, s) != hipSuccess) {
            fail(AH_E_HIP);
            return;
        }
        S.busy = true;
    }

    void wait(int i) {
        Slot &S = slot[i];
        if (S.busy && hipEventSynchronize(S.ev) != hipSuccess) fail(AH_E_HIP);
        S.busy = false;
    }

    // Send slot[cur] to the GPU and continue in the other slot.  An open
    // piece keeps whole blocks; its last (len mod 64) bases move to the new
    // slot as the start of the record's next piece.
    void flush() {
        Slot &S = slot[cur];
        uint32_t t = 0;
        if (piece >= 0) {
            ah_pack_piece &P = S.h_pcs[piece];
            t = P.n & 63u;
            P.n -= t;
            if (P.n == 0) S.npcs--;
        }
        S.nbytes -= t;
        const uint8_t *tail = S.h_buf + S.nbytes;
        submit(cur);
        cur ^= 1;
        wait(cur);
        Slot &T = slot[cur];
        T.nbytes = 0;
        T.npcs = 0;
        piece = -1;
        if (t) {
            T.h_pcs[0] = ah_pack_piece{0, rec_block0 + (rec_len - t) / 64, t, 0};
            T.npcs = 1;
            piece = 0;
            memcpy(T.h_buf, tail, t);
            T.nbytes = t;
        }
    }

    void add_bases(const uint8_t *p, size_t n) {
        if (!device) {
            rec_len += count_bases(p, n);
            return;
        }
        while (n && !err) {
            Slot &S = slot[cur];
            const uint64_t room = chunk - S.nbytes;
            if (room == 0 || (piece < 0 && S.npcs == pcap)) {
                flush();
                continue;
            }
            if (piece < 0) {  // rec_len is a multiple of 64 here
                S.h_pcs[S.npcs] = ah_pack_piece{S.nbytes, rec_block0 + rec_len / 64, 0, 0};
                piece = S.npcs++;
            }
            const size_t m = n < room ? n : (size_t)room;
            const size_t k = copy_bases(S.h_buf + S.nbytes, p, m);
            S.nbytes += k;
            S.h_pcs[piece].n += (uint32_t)k;
            rec_len += k;
            p += m;
            n -= m;
        }
    }

    // Parse one file.
    ah_status file(const char *path, uint32_t fi, uint8_t *rb) {
        int fd = open(path, O_RDONLY | O_CLOEXEC);
        if (fd < 0) return AH_E_IO;
        posix_fadvise(fd, 0, 0, POSIX_FADV_SEQUENTIAL);
        enum { kLineStart, kBeforeFirst, kIdSkip, kId, kHeaderRest, kSeq } st = kLineStart;
        bool seen_header = false;
        ah_status ret = AH_OK;
        for (;;) {
            ssize_t got = read(fd, rb, kReadBytes);
            if (got < 0) {
                if (errno == EINTR) continue;
                ret = AH_E_IO;
                break;
            }
            if (got == 0) break;
            const uint8_t *p = rb, *e = rb + got;
            while (p < e && !err && !ret) {
                switch (st) {
                case kLineStart:
                    if (*p == '>') {
                        if (in_rec) end_record();
                        begin_record(fi);
                        seen_header = true;
                        st = kIdSkip;
                        p++;
                    } else {
                        st = seen_header ? kSeq : kBeforeFirst;
                    }
                    break;
                case kBeforeFirst: {  // only white space may precede the first header
                    const uint8_t *nl = (const uint8_t *)memchr(p, '\n', e - p);
                    const uint8_t *q = nl ? nl : e;
                    for (; p < q; p++)
                        if (!kSpace.t[*p]) ret = AH_E_FORMAT;
                    if (nl) {
                        p = nl + 1;
                        st = kLineStart;
                    }
                    break;
                }
                case kIdSkip:  // white space before the identifier
                    if (*p == '\n') {
                        st = kLineStart;
                        p++;
                    } else if (kSpace.t[*p]) {
                        p++;
                    } else {
                        st = kId;
                    }
                    break;
                case kId: {
                    const uint8_t *q = p;
                    while (q < e && !kSpace.t[*q]) q++;
                    f->ids.append((const char *)p, q - p);
                    p = q;
                    if (q < e) st = kHeaderRest;
                    break;
                }
                case kHeaderRest: {
                    const uint8_t *nl = (const uint8_t *)memchr(p, '\n', e - p);
                    if (nl) {
                        p = nl + 1;
                        st = kLineStart;
                    } else {
                        p = e;
                    }
                    break;
                }
                case kSeq: {
                    const uint8_t *nl = (const uint8_t *)memchr(p, '\n', e - p);
                    const uint8_t *q = nl ? nl : e;
                    add_bases(p, q - p);
                    if (nl) {
                        p = nl + 1;
                        st = kLineStart;
                    } else {
                        p = e;
                    }
                    break;
                }
                }
            }
            if (err || ret) break;
        }
        close(fd);
        if (!ret && !err && in_rec) end_record();
        return ret ? ret : err;
    }
};

std::string base_name(const char *path) {
    const char *b = strrchr(path, '/');
    return std::string(b ? b + 1 : path);
}

}  // namespace

extern "C" ah_status ah_fasta_ws_size(uint64_t chunk_bytes, uint64_t *bytes) {
    if (!bytes || chunk_bytes < 4096 || chunk_bytes > (1ull << 30)) return AH_E_ARG;
    *bytes = 2 * (ah_align_up(chunk_bytes, 256) + ah_align_up(pieces_per_chunk(chunk_bytes) * sizeof(ah_pack_piece), 256));
    return AH_OK;
}

namespace {

struct Target {  // where and how a worker packs
    uint64_t chunk;
    uint8_t *d_ws;   // this worker's device staging (ah_fasta_ws_size bytes)
    hipStream_t s;
    uint32_t *d_blocks;
    uint64_t blocks_cap;
    uint32_t *d_nbits;
    uint64_t *d_counters;
    uint64_t *d_nlist;
    uint64_t nlist_cap;
};

// Set up g for packing into t (pinned staging allocated here).
ah_status ingest_open(Ingest &g, const Target &t) {
    g.device = true;
    g.chunk = t.chunk;
    g.pcap = (uint32_t)pieces_per_chunk(t.chunk);
    g.s = t.s;
    g.d_blocks = t.d_blocks;
    g.blocks_cap = t.blocks_cap;
    g.d_nbits = t.d_nbits;
    g.d_counters = t.d_counters;
    g.d_nlist = t.d_nlist;
    g.nlist_cap = t.nlist_cap;
    const uint64_t a = ah_align_up(g.chunk, 256), b = ah_align_up((uint64_t)g.pcap * sizeof(ah_pack_piece), 256);
    for (int i = 0; i < 2; i++) {
        Slot &S = g.slot[i];
        S.d_buf = t.d_ws + i * (a + b);
        S.d_pcs = (ah_pack_piece *)(t.d_ws + i * (a + b) + a);
        if (hipHostMalloc((void **)&S.h_buf, g.chunk, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&S.h_pcs, (uint64_t)g.pcap * sizeof(ah_pack_piece), hipHostMallocDefault) !=
                hipSuccess ||
            hipEventCreateWithFlags(&S.ev, hipEventDisableTiming) != hipSuccess)
            return AH_E_HIP;
    }
    return AH_OK;
}

// Send what is staged, wait for both slots, free the staging.
ah_status ingest_close(Ingest &g, ah_status ret) {
    if (!ret) g.submit(g.cur);
    g.wait(0);
    g.wait(1);
    if (!ret) ret = g.err;
    for (int i = 0; i < 2; i++) {
        Slot &S = g.slot[i];
        if (S.h_buf && hipHostFree(S.h_buf) != hipSuccess && !ret) ret = AH_E_HIP;
        if (S.h_pcs && hipHostFree(S.h_pcs) != hipSuccess && !ret) ret = AH_E_HIP;
        if (S.ev && hipEventDestroy(S.ev) != hipSuccess && !ret) ret = AH_E_HIP;
        S.h_buf = nullptr;
        S.h_pcs = nullptr;
        S.ev = nullptr;
    }
    return ret;
}

// Run fn(worker) on n host threads (inline when n == 1); first error wins.
template <class Fn>
ah_status run_workers(uint32_t n, Fn fn) {
    std::vector<ah_status> st(n, AH_OK);
    if (n == 1) {
        st[0] = fn(0u);
    } else {
        std::vector<std::thread> th;
        for (uint32_t w = 0; w < n; w++) th.emplace_back([&, w] { st[w] = fn(w); });
        for (auto &t : th) t.join();
    }
    for (ah_status e : st)
        if (e) return e;
    return AH_OK;
}

// Append part's records (one file, blocks numbered from 0) to f.
void append_part(ah_fasta *f, const ah_fasta &part) {
    const uint64_t base = f->n_blocks, id0 = f->ids.size();
    for (size_t r = 0; r < part.len.size(); r++) {
        f->len.push_back(part.len[r]);
        f->block0.push_back(base + part.block0[r]);
        f->file.push_back(part.file[r]);
        f->id_off.push_back(id0 + part.id_off[r]);
    }
    f->ids.append(part.ids);
    f->n_blocks += part.n_blocks;
    f->n_bases += part.n_bases;
    if (part.max_len > f->max_len) f->max_len = part.max_len;
}

}  // namespace

extern "C" ah_status ah_fasta_ingest(const char *const *paths, uint32_t n_files, uint32_t *d_blocks,
                                     uint64_t blocks_cap, uint32_t *d_nbits, uint64_t *d_counters, uint64_t *d_nlist,
                                     uint64_t nlist_cap, uint64_t chunk_bytes, uint32_t n_threads, void *d_ws,
                                     uint64_t ws_bytes, void *stream, ah_fasta **out) {
    if (!out || (n_files && !paths)) return AH_E_ARG;
    for (uint32_t i = 0; i < n_files; i++)
        if (!paths[i]) return AH_E_ARG;
    const bool device = d_blocks != nullptr;
    uint32_t workers = n_threads ? n_threads : 1;
    if (workers > n_files) workers = n_files ? n_files : 1;
    if (workers > 64) workers = 64;
    uint64_t per_ws = 0;
    if (device) {
        if (ah_fasta_ws_size(chunk_bytes, &per_ws)) return AH_E_ARG;
        if (!d_nbits || !d_counters || (nlist_cap && !d_nlist) || !d_ws) return AH_E_ARG;
        if (ws_bytes < per_ws) return AH_E_WORKSPACE;
        if (ws_bytes < per_ws * workers) workers = (uint32_t)(ws_bytes / per_ws);  // as many as the workspace holds
    }
    Target t{chunk_bytes, (uint8_t *)d_ws, ah_stream(stream), d_blocks, blocks_cap, d_nbits, d_counters, d_nlist,
             nlist_cap};
    ah_fasta *f = new ah_fasta();
    for (uint32_t i = 0; i < n_files; i++) f->files.push_back(base_name(paths[i]));
    ah_status ret = AH_OK;
    if (device) {
        ah_fill<uint32_t>(d_nbits, 0u, (blocks_cap + 31) / 32, t.s);
        ah_fill<uint64_t>(d_counters, 0ull, AH_STORE_SCRATCH, t.s);
        if (hipGetLastError() != hipSuccess) ret = AH_E_HIP;
    }
    if (!ret && workers <= 1) {
        // one pass: parse, stage and pack every file in order
        Ingest g;
        g.f = f;
        std::vector<uint8_t> rb(kReadBytes);
        if (device) ret = ingest_open(g, t);
        for (uint32_t i = 0; i < n_files && !ret; i++) ret = g.file(paths[i], i, rb.data());
        if (device) ret = ingest_close(g, ret);
    } else if (!ret) {
        // index every file in parallel, fix the layout in file order, pack in parallel
        std::vector<ah_fasta> parts(n_files);
        std::atomic<uint32_t> next{0};
        ret = run_workers(workers, [&](uint32_t) -> ah_status {
            std::vector<uint8_t> rb(kReadBytes);
            for (uint32_t i; (i = next.fetch_add(1)) < n_files;) {
                Ingest g;
                g.f = &parts[i];
                const ah_status e = g.file(paths[i], i, rb.data());
                if (e) return e;
            }
            return AH_OK;
        });
        std::vector<uint64_t> base(n_files, 0);
        for (uint32_t i = 0; i < n_files && !ret; i++) {
            base[i] = f->n_blocks;
            append_part(f, parts[i]);
            if (f->len.size() >= 0xFFFFFFFFull) ret = AH_E_FORMAT;
        }
        if (!ret && device) {
            std::atomic<uint32_t> next2{0};
            ret = run_workers(workers, [&](uint32_t w) -> ah_status {
                Target tw = t;
                tw.d_ws = t.d_ws + (uint64_t)w * per_ws;
                Ingest g;
                std::vector<uint8_t> rb(kReadBytes);
                ah_status e = ingest_open(g, tw);
                for (uint32_t i; !e && (i = next2.fetch_add(1)) < n_files;) {
                    ah_fasta scratch;
                    scratch.n_blocks = base[i];  // records numbered from the file's first block
                    g.f = &scratch;
                    e = g.file(paths[i], i, rb.data());
                    if (!e && scratch.n_blocks - base[i] != parts[i].n_blocks) e = AH_E_IO;  // file changed
                }
                return ingest_close(g, e);
            });
        }
    }
    if (device && hipStreamSynchronize(t.s) != hipSuccess && !ret) ret = AH_E_HIP;
    if (ret) {
        delete f;
        return ret;
    }
    for (const std::string &x : f->files) f->file_ptrs.push_back(x.c_str());
    *out = f;
    return AH_OK;
}

extern "C" ah_status ah_fasta_info(const ah_fasta *f, uint32_t *n_records, uint64_t *n_bases, uint64_t *n_blocks,
                                   uint32_t *max_len) {
    if (!f) return AH_E_ARG;
    if (n_records) *n_records = (uint32_t)f->len.size();
    if (n_bases) *n_bases = f->n_bases;
    if (n_blocks) *n_blocks = f->n_blocks;
    if (max_len) *max_len = f->max_len;
    return AH_OK;
}

extern "C" ah_status ah_fasta_table(const ah_fasta *f, uint32_t *h_len, uint64_t *h_block0) {
    if (!f || (!f->len.empty() && (!h_len || !h_block0))) return AH_E_ARG;
    if (!f->len.empty()) {
        memcpy(h_len, f->len.data(), f->len.size() * sizeof(uint32_t));
        memcpy(h_block0, f->block0.data(), f->block0.size() * sizeof(uint64_t));
    }
    return AH_OK;
}

extern "C" ah_status ah_fasta_names_of(const ah_fasta *f, ah_fasta_names *out) {
    if (!f || !out) return AH_E_ARG;
    out->ids = f->ids.data();
    out->id_off = f->id_off.data();
    out->seq_file = f->file.data();
    out->files = f->file_ptrs.data();
    out->n_seqs = (uint32_t)f->len.size();
    out->n_files = (uint32_t)f->files.size();
    return AH_OK;
}

extern "C" void ah_fasta_free(ah_fasta *f) { delete f; }

// ---------------------------------------------------------------- output
namespace {

struct Out {
    char *buf;
    uint64_t cap;
    uint64_t pos = 0;
    void put(const char *p, uint64_t n) {
        if (pos < cap) memcpy(buf + pos, p, n < cap - pos ? n : cap - pos);
        pos += n;
    }
    void put(const char *z) { put(z, strlen(z)); }
};

uint64_t strnlen32(const char *p) {
    uint64_t n = 0;
    while (n < 32 && p[n]) n++;
    return n;
}

}  // namespace

// Records in FASTA (">" header, bases) or, with h_qual, FASTQ ("@" header,
// bases, "+", qualities).
static ah_status format_records(const ah_fasta_names *nm, uint32_t fb_len, uint32_t rb_len, const ah_amp *h_amps,
                                uint64_t n_amps, const double *h_tm, const uint8_t *h_pass, const char *h_seq,
                                const uint64_t *h_seq_off, const char *h_qual, const char *h_fb, const char *h_rb,
                                const uint8_t *h_bc_len, const char *h_fprimer, const char *h_rprimer, char *h_out,
                                uint64_t out_cap, uint64_t *h_n_bytes, bool fastq) {
    if (!nm || !h_n_bytes || (out_cap && !h_out)) return AH_E_ARG;
    if (n_amps && (!h_amps || !h_tm || !h_seq_off || !h_bc_len || !h_fprimer || !h_rprimer)) return AH_E_ARG;
    if (n_amps && (!nm->ids || !nm->id_off || !nm->seq_file || !nm->files)) return AH_E_ARG;
    if ((fb_len && !h_fb) || (rb_len && !h_rb) || fb_len > 255 || rb_len > 255) return AH_E_ARG;
    // validate everything before writing
    for (uint64_t i = 0; i < n_amps; i++) {
        const ah_amp &a = h_amps[i];
        if (a.seq >= nm->n_seqs || nm->seq_file[a.seq] >= nm->n_files || a.orient > 3) return AH_E_ARG;
        if (h_seq_off[i + 1] < h_seq_off[i] || h_bc_len[2 * i] > fb_len || h_bc_len[2 * i + 1] > rb_len)
            return AH_E_ARG;
        if (h_seq_off[i + 1] > h_seq_off[i] && (!h_seq || (fastq && !h_qual))) return AH_E_ARG;
    }
    static const char *kOrient[4] = {"FR", "RF", "FF", "RR"};
    Out o{h_out, out_cap};
    char num[64];
    for (uint64_t i = 0; i < n_amps; i++) {
        if (h_pass && !h_pass[i]) continue;
        const ah_amp &a = h_amps[i];
        o.put(fastq ? "@" : ">");
        o.put(nm->ids + nm->id_off[a.seq]);
        o.put(".source=");
        o.put(nm->files[nm->seq_file[a.seq]]);
        snprintf(num, sizeof num, ".coordinates=%llu-%llu.Tm=", (unsigned long long)a.start + 1ull,
                 (unsigned long long)a.end);
        o.put(num);
        if (std::isfinite(h_tm[i])) {
            snprintf(num, sizeof num, "%.2f", h_tm[i]);
            o.put(num);
        } else {
            o.put("NA");
        }
        o.put(".orientation=");
        o.put(kOrient[a.orient]);
        o.put(".fprimer=");
        o.put(h_fprimer + 32 * i, strnlen32(h_fprimer + 32 * i));
        o.put(".rprimer=");
        o.put(h_rprimer + 32 * i, strnlen32(h_rprimer + 32 * i));
        if (fb_len) {
            o.put(".fb=");
            o.put(h_fb + (uint64_t)fb_len * i, h_bc_len[2 * i]);
        }
        if (rb_len) {
            o.put(".rb=");
            o.put(h_rb + (uint64_t)rb_len * i, h_bc_len[2 * i + 1]);
        }
        o.put("\n");
        o.put(h_seq + h_seq_off[i], h_seq_off[i + 1] - h_seq_off[i]);
        o.put("\n");
        if (fastq) {
            o.put("+\n");
            o.put(h_qual + h_seq_off[i], h_seq_off[i + 1] - h_seq_off[i]);
            o.put("\n");
        }
    }
    *h_n_bytes = o.pos;
    return AH_OK;
}

extern "C" ah_status ah_fasta_format(const ah_fasta_names *nm, uint32_t fb_len, uint32_t rb_len, const ah_amp *h_amps,
                                     uint64_t n_amps, const double *h_tm, const uint8_t *h_pass, const char *h_seq,
                                     const uint64_t *h_seq_off, const char *h_fb, const char *h_rb,
                                     const uint8_t *h_bc_len, const char *h_fprimer, const char *h_rprimer,
                                     char *h_out, uint64_t out_cap, uint64_t *h_n_bytes) {
    return format_records(nm, fb_len, rb_len, h_amps, n_amps, h_tm, h_pass, h_seq, h_seq_off, nullptr, h_fb, h_rb,
                          h_bc_len, h_fprimer, h_rprimer, h_out, out_cap, h_n_bytes, false);
}

extern "C" ah_status ah_fastq_format(const ah_fasta_names *nm, uint32_t fb_len, uint32_t rb_len, const ah_amp *h_amps,
                                     uint64_t n_amps, const double *h_tm, const uint8_t *h_pass, const char *h_seq,
                                     const uint64_t *h_seq_off, const char *h_qual, const char *h_fb,
                                     const char *h_rb, const uint8_t *h_bc_len, const char *h_fprimer,
                                     const char *h_rprimer, char *h_out, uint64_t out_cap, uint64_t *h_n_bytes) {
    return format_records(nm, fb_len, rb_len, h_amps, n_amps, h_tm, h_pass, h_seq, h_seq_off, h_qual, h_fb, h_rb,
                          h_bc_len, h_fprimer, h_rprimer, h_out, out_cap, h_n_bytes, true);
}
