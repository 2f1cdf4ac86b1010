// Autotuner: per (operation, shape bucket) the fastest of a few equivalent
// schedules, measured once on the live data with HIP events and kept in the
// context's table.  Every candidate of an operation computes the same result
// (the triangular solve's rows per tile, the radix sort's digit width and
// tile size), so a choice affects time only and never an output.
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.hpp"

u64 tune_key(TuneOp op, u32 a, u32 b, u32 c) {
    return ((u64)op << 48) | ((u64)(a & 0xffffu) << 32) | ((u64)(b & 0xffffu) << 16) | (u64)(c & 0xffffu);
}

u32 tune_lg(u64 x) {
    u32 l = 0;
    while (((u64)1 << l) < x) ++l;
    return l;
}

u32 tune_pick(Ctx& c, u64 key, const std::vector<u32>& cands, const std::function<void(u32)>& prep,
              const std::function<void(u32)>& run) {
    if (cands.empty()) throw F4Error{1, "autotuner: no candidate"};
    auto it = c.tune.table.find(key);
    if (it != c.tune.table.end())
        for (u32 v : cands)
            if (v == it->second) return v;
    if (cands.size() == 1) {
        c.tune.table[key] = cands[0];
        return cands[0];
    }
    const int reps = 2;
    const size_t ne = 2 * cands.size() * reps;
    std::vector<hipEvent_t> ev(ne, nullptr);
    std::vector<float> best(cands.size(), 3.0e38f);
    try {
        for (auto& e : ev) F4_HIP_TRY(hipEventCreate(&e));
        size_t k = 0;
        for (int r = 0; r < reps; ++r)
            for (size_t i = 0; i < cands.size(); ++i) {
                prep(cands[i]);
                F4_HIP_TRY(hipEventRecord(ev[k], c.stream));
                run(cands[i]);
                F4_HIP_TRY(hipEventRecord(ev[k + 1], c.stream));
                k += 2;
            }
        F4_HIP_TRY(hipEventSynchronize(ev[ne - 1]));
        k = 0;
        for (int r = 0; r < reps; ++r)
            for (size_t i = 0; i < cands.size(); ++i) {
                float ms = 0.f;
                F4_HIP_TRY(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
                if (ms < best[i]) best[i] = ms;
                k += 2;
            }
    } catch (...) {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        throw;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    size_t bi = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (best[i] < best[bi]) bi = i;
    c.tune.table[key] = cands[bi];
    return cands[bi];
}

// Text form of the table, one entry per line:
//   trsm <small> <lg2 rows> <lg2 N> <rows per tile>
//   sort <with values> <lg2 n> <key bits> <digit bits> <keys per thread>
std::string tune_text(const Ctx& c) {
    std::string out;
    char line[96];
    for (const auto& kv : c.tune.table) {
        const u32 op = (u32)(kv.first >> 48), a = (u32)(kv.first >> 32) & 0xffffu,
                  b = (u32)(kv.first >> 16) & 0xffffu, d = (u32)kv.first & 0xffffu;
        if (op == TUNE_TRSM)
            snprintf(line, sizeof line, "trsm %u %u %u %u\n", a, b, d, kv.second);
        else if (op == TUNE_SORT)
            snprintf(line, sizeof line, "sort %u %u %u %u %u\n", a, b, d, kv.second & 0xffu, kv.second >> 8);
        else
            continue;
        out += line;
    }
    return out;
}

// Parses the text form; entries are checked for range and merged into the
// table (a later entry for the same bucket wins).  Throws on a malformed line.
void tune_parse(Ctx& c, const char* text) {
    std::map<u64, u32> add;
    const char* p = text;
    while (*p) {
        const char* e = strchr(p, '\n');
        const size_t len = e ? (size_t)(e - p) : strlen(p);
        std::string ln(p, len);
        p += len + (e ? 1 : 0);
        if (ln.find_first_not_of(" \t\r") == std::string::npos) continue;
        unsigned a, b, d, v, w;
        char tail;
        if (sscanf(ln.c_str(), "trsm %u %u %u %u %c", &a, &b, &d, &v, &tail) == 4) {
            if (a > 1 || b > 64 || d > 64 || v < 1 || v > 4) throw F4Error{1, "tune table: bad trsm entry: " + ln};
            add[tune_key(TUNE_TRSM, a, b, d)] = v;
        } else if (sscanf(ln.c_str(), "sort %u %u %u %u %u %c", &a, &b, &d, &v, &w, &tail) == 5) {
            if (a > 1 || b > 64 || d > 64 || v < 1 || v > 8 || w < 1 || w > 64)
                throw F4Error{1, "tune table: bad sort entry: " + ln};
            add[tune_key(TUNE_SORT, a, b, d)] = v | (w << 8);
        } else {
            throw F4Error{1, "tune table: unreadable line: " + ln};
        }
    }
    for (const auto& kv : add) c.tune.table[kv.first] = kv.second;
}
