// Record table of FASTA or FASTQ input (host memory owned by libah.so):
// identifiers, source files, lengths and first blocks in the store layout
// (each record starts on a new 64-base block).  FASTQ input also keeps its
// records' bases and qualities, back to back.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

struct ah_fasta {
    std::vector<std::string> files;   // source names (path without directories)
    std::vector<const char *> file_ptrs;
    std::vector<uint32_t> len;
    std::vector<uint64_t> block0;
    std::vector<uint32_t> file;
    std::vector<uint64_t> id_off;
    std::string ids;                  // NUL-terminated identifiers, back to back
    uint64_t n_bases = 0;
    uint64_t n_blocks = 0;
    uint32_t max_len = 0;
    // FASTQ only: record r's bases and qualities are [off[r], off[r + 1]) of
    // bases / qual
    bool fastq = false;
    std::string bases, qual;
    std::vector<uint64_t> off;
};
