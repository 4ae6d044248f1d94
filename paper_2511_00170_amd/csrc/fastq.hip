// FASTQ input with quality propagation (host code).  The paper's Discussion
// names FASTQ input with qualities carried to the amplicons as the step that
// makes the engine usable on amplicon sequencing reads; the Python AHv1.1
// reads FASTQ (--input-fq).
//
// A file is read whole and parsed into the record table of the FASTA path
// (identifiers, sources, lengths, store layout) plus the bases and qualities
// of every record, back to back.  The bases then go through the ordinary
// pack call; the qualities are laid out like the store's bases (record r's
// quality of base j at byte 64 * block0[r] + j) so that the extraction
// kernels read a base's quality at the base's own store position.
#include <errno.h>
#include <fcntl.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <string>

#include "ah.h"
#include "ah_internal.h"
#include "fasta_table.h"

namespace {

// White space inside a header line: space, tab, VT, FF (CR only ends a line).
inline bool header_space(char c) { return c == ' ' || c == '\t' || c == '\v' || c == '\f' || c == '\r'; }

ah_status read_file(const char *path, std::string &buf) {
    int fd = open(path, O_RDONLY | O_CLOEXEC);
    if (fd < 0) return AH_E_IO;
    struct stat sb;
    if (fstat(fd, &sb) != 0) {
        close(fd);
        return AH_E_IO;
    }
    buf.resize((size_t)sb.st_size);
    size_t got = 0;
    while (got < buf.size()) {
        const ssize_t r = read(fd, &buf[got], buf.size() - got);
        if (r < 0 && errno == EINTR) continue;
        if (r <= 0) {
            close(fd);
            return AH_E_IO;
        }
        got += (size_t)r;
    }
    char extra;
    const ssize_t r = read(fd, &extra, 1);  // the file grew while being read
    close(fd);
    return r == 0 ? AH_OK : AH_E_IO;
}

// Line [s, e) starting at i (without its LF and a CR before it); false at the
// end of the text.
inline bool next_line(const std::string &b, size_t &i, size_t &s, size_t &e) {
    if (i >= b.size()) return false;
    s = i;
    const char *nl = (const char *)memchr(b.data() + i, '\n', b.size() - i);
    e = nl ? (size_t)(nl - b.data()) : b.size();
    i = nl ? e + 1 : b.size();
    if (e > s && b[e - 1] == '\r') e--;
    return true;
}

// Records of one file: "@header" / bases / "+..." / qualities, four lines
// each; empty lines between records are skipped.  The identifier is the
// header's first white-space-separated word; qualities are bytes '!'..'~',
// exactly one per base.
ah_status parse(const std::string &b, uint32_t fi, ah_fasta *f) {
    size_t i = 0, s, e;
    while (next_line(b, i, s, e)) {
        if (s == e) continue;
        if (b[s] != '@') return AH_E_FORMAT;
        size_t a = s + 1;
        while (a < e && header_space(b[a])) a++;
        size_t z = a;
        while (z < e && !header_space(b[z])) z++;
        size_t bs, be, ps, pe, qs, qe;
        if (!next_line(b, i, bs, be) || !next_line(b, i, ps, pe) || !next_line(b, i, qs, qe)) return AH_E_FORMAT;
        if (pe == ps || b[ps] != '+') return AH_E_FORMAT;
        const uint64_t L = be - bs;
        if (qe - qs != L || L >= (1ull << 32) || f->len.size() >= 0xFFFFFFFFull) return AH_E_FORMAT;
        for (size_t k = qs; k < qe; k++)
            if ((unsigned char)b[k] < '!' || (unsigned char)b[k] > '~') return AH_E_FORMAT;
        for (size_t k = bs; k < be; k++)
            if ((unsigned char)b[k] <= ' ' || (unsigned char)b[k] > '~') return AH_E_FORMAT;
        f->id_off.push_back(f->ids.size());
        f->ids.append(b, a, z - a);
        f->ids.push_back('\0');
        f->file.push_back(fi);
        f->len.push_back((uint32_t)L);
        f->block0.push_back(f->n_blocks);
        f->n_blocks += (L + 63) / 64;
        f->n_bases += L;
        if (L > f->max_len) f->max_len = (uint32_t)L;
        f->bases.append(b, bs, L);
        f->qual.append(b, qs, L);
        f->off.push_back(f->bases.size());
    }
    return AH_OK;
}

}  // namespace

extern "C" ah_status ah_fastq_read(const char *const *paths, uint32_t n_files, ah_fasta **out) {
    if (!out || (n_files && !paths)) return AH_E_ARG;
    for (uint32_t k = 0; k < n_files; k++)
        if (!paths[k]) return AH_E_ARG;
    ah_fasta *f = new ah_fasta;
    f->fastq = true;
    f->off.push_back(0);
    std::string buf;
    for (uint32_t k = 0; k < n_files; k++) {
        const char *sl = strrchr(paths[k], '/');
        f->files.push_back(std::string(sl ? sl + 1 : paths[k]));
        ah_status e = read_file(paths[k], buf);
        if (!e) e = parse(buf, k, f);
        if (e) {
            delete f;
            return e;
        }
    }
    for (const std::string &x : f->files) f->file_ptrs.push_back(x.c_str());
    *out = f;
    return AH_OK;
}

extern "C" ah_status ah_fastq_bases(const ah_fasta *f, const char **h_bases, const uint64_t **h_off) {
    if (!f || !f->fastq || !h_bases || !h_off) return AH_E_ARG;
    *h_bases = f->bases.data();
    *h_off = f->off.data();
    return AH_OK;
}

extern "C" ah_status ah_fastq_qual_layout(const ah_fasta *f, uint8_t *h_qual, uint64_t cap) {
    if (!f || !f->fastq || (cap && !h_qual)) return AH_E_ARG;
    if (cap < 64 * f->n_blocks) return AH_E_LIMIT;
    memset(h_qual, 0, cap);
    for (size_t r = 0; r < f->len.size(); r++)
        memcpy(h_qual + 64 * f->block0[r], f->qual.data() + f->off[r], f->len[r]);
    return AH_OK;
}
