// Tuning cache of the uneven-batch plan: a flat JSON object
// {"key": [block, blocks_per_cu, px_per_lane], ...} mapping a problem class to the fastest
// launch shape found for it (an entry without the third value means 4 pixels per lane).
// Host code only (no HIP), so that a CPU build can exercise the parser on its own.
#pragma once

#include <cctype>
#include <cstdlib>
#include <map>
#include <string>

namespace svdlut {

struct TuneEntry {
    int block;    // threads per workgroup: 64, 128, 256, 512 or 1024
    int bpc;      // workgroups per CU in the persistent launch: 1 .. 32
    int px = 4;   // pixels per lane (tile width 64 * px): 4 or 8
};

inline bool tune_entry_ok(const TuneEntry& e) {
    return (e.block == 64 || e.block == 128 || e.block == 256 || e.block == 512 || e.block == 1024) && e.bpc >= 1 &&
           e.bpc <= 32 && (e.px == 4 || e.px == 8);
}

namespace tune_detail {

inline void skip_ws(const std::string& t, size_t& i) {
    while (i < t.size() && std::isspace(static_cast<unsigned char>(t[i]))) ++i;
}

// a decimal integer of at most 9 digits (optional sign) at t[i]; false if there is none
inline bool read_int(const std::string& t, size_t& i, int& v) {
    size_t j = i;
    bool neg = false;
    if (j < t.size() && (t[j] == '-' || t[j] == '+')) neg = t[j++] == '-';
    const size_t d0 = j;
    long acc = 0;
    while (j < t.size() && std::isdigit(static_cast<unsigned char>(t[j])) && j - d0 < 9) acc = acc * 10 + (t[j++] - '0');
    if (j == d0 || (j < t.size() && std::isdigit(static_cast<unsigned char>(t[j])))) return false;
    v = static_cast<int>(neg ? -acc : acc);
    i = j;
    return true;
}

}  // namespace tune_detail

// Adds every well-formed entry of `txt` with valid values to `out` (later duplicates win) and
// returns how many it accepted.  Anything else (truncation, wrong types, out-of-range
// values, other JSON) is skipped; nothing is read outside the string.
inline int parse_tune_cache(const std::string& txt, std::map<std::string, TuneEntry>& out) {
    using namespace tune_detail;
    int n = 0;
    size_t pos = 0;
    while (pos < txt.size()) {
        const size_t k0 = txt.find('"', pos);
        if (k0 == std::string::npos) break;
        const size_t k1 = txt.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        pos = k1 + 1;
        size_t i = k1 + 1;
        skip_ws(txt, i);
        if (i >= txt.size() || txt[i] != ':') continue;
        ++i;
        skip_ws(txt, i);
        if (i >= txt.size() || txt[i] != '[') continue;
        ++i;
        TuneEntry e{0, 0, 4};
        skip_ws(txt, i);
        if (!read_int(txt, i, e.block)) continue;
        skip_ws(txt, i);
        if (i >= txt.size() || txt[i] != ',') continue;
        ++i;
        skip_ws(txt, i);
        if (!read_int(txt, i, e.bpc)) continue;
        skip_ws(txt, i);
        if (i < txt.size() && txt[i] == ',') {   // optional third value: pixels per lane
            ++i;
            skip_ws(txt, i);
            if (!read_int(txt, i, e.px)) continue;
            skip_ws(txt, i);
        }
        if (i >= txt.size() || txt[i] != ']') continue;
        pos = i + 1;
        if (!tune_entry_ok(e) || k1 - k0 - 1 > 512) continue;
        out[txt.substr(k0 + 1, k1 - k0 - 1)] = e;
        ++n;
    }
    return n;
}

inline std::string format_tune_cache(const std::map<std::string, TuneEntry>& m) {
    std::string s = "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
        s += "  \"" + kv.first + "\": [" + std::to_string(kv.second.block) + ", " + std::to_string(kv.second.bpc) +
             ", " + std::to_string(kv.second.px) + "]" + (++i < m.size() ? "," : "") + "\n";
    }
    s += "}\n";
    return s;
}

}  // namespace svdlut
