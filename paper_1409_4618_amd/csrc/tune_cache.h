// The batch autotuner's cache file: plain host code, shared by the library and
// the host-only sanitizer check of its parsing.
//
// One JSON object per line,
//   {"device": "...", "signature": "...", "rows_per_tile": R, "schedule": S, "threads": N, "ms": t}
// A lookup takes the last line whose device and signature match and whose
// rows per tile (0, 64, 128, 256), schedule (0-4 for element-major tiles,
// 0-2 for row tiles) and threads (128 or 256 for element-major tiles, 256 for
// row tiles; 256 when the field is absent) are valid; malformed, truncated or foreign lines are skipped. A store appends
// one line.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>

namespace fem {

// Parses a decimal integer of at most 9 digits after `key` in `line`; false if
// the key is absent or no digits follow it.
inline bool cache_field(const std::string& line, const char* key, int* out) {
    const size_t p = line.find(key);
    if (p == std::string::npos) return false;
    size_t i = p + std::char_traits<char>::length(key);
    bool neg = false;
    if (i < line.size() && line[i] == '-') {
        neg = true;
        ++i;
    }
    int v = 0, nd = 0;
    while (i < line.size() && line[i] >= '0' && line[i] <= '9' && nd < 9) {
        v = v * 10 + (line[i] - '0');
        ++i;
        ++nd;
    }
    if (nd == 0) return false;
    *out = neg ? -v : v;
    return true;
}

inline bool cache_lookup(const char* path, const std::string& dev, const std::string& sig, int* R,
                         int* sched, int* threads) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    const std::string kd = "\"device\": \"" + dev + "\"";
    const std::string ks = "\"signature\": \"" + sig + "\"";
    while (std::getline(f, line)) {
        if (line.find(kd) == std::string::npos) continue;
        if (line.find(ks) == std::string::npos) continue;
        int r = -1, sc = -1, nt = 256;
        if (!cache_field(line, "\"rows_per_tile\": ", &r) || !cache_field(line, "\"schedule\": ", &sc))
            continue;
        if (line.find("\"threads\": ") != std::string::npos && !cache_field(line, "\"threads\": ", &nt))
            continue;
        const bool nt_ok = r == 0 ? (nt == 128 || nt == 256) : nt == 256;
        if ((r == 0 || r == 64 || r == 128 || r == 256) && sc >= 0 && sc <= (r == 0 ? 4 : 2) && nt_ok) {
            *R = r;
            *sched = sc;
            *threads = nt;
            found = true;  // last matching line wins
        }
    }
    return found;
}

inline void cache_store(const char* path, const std::string& dev, const std::string& sig, int R, int sched,
                        int threads, double ms) {
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    // device and signature are written as given (the library builds both from
    // characters that need no JSON escaping); the line length is not bounded
    // by a fixed buffer
    f << "{\"device\": \"" << dev << "\", \"signature\": \"" << sig << "\", \"rows_per_tile\": " << R
      << ", \"schedule\": " << sched << ", \"threads\": " << threads << ", \"ms\": ";
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%.6f", ms);
    f << buf << "}\n";
}

}  // namespace fem
