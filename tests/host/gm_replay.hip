// Host-only replay of the pair-set updates along a leading-monomial insertion
// sequence: the generic Gebauer-Moeller update and the fast one run side by
// side and must hold the same pair set after every insertion; a third state
// inserts each step's elements at once (gm_insert_step) and must agree with
// them at every step boundary; there the pairs of least degree are selected
// and counted.
//
// Input (text): n, then lines "I a_1 .. a_n" (insert an element with this
// leading monomial) and "S d nsel" (select; expect nsel pairs of degree d).
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "../../paper_2601_06765_amd/csrc/pairs.hpp"

static std::vector<std::pair<u64, u64>> as_set(const std::vector<HPair>& P) {
    std::vector<std::pair<u64, u64>> s;
    for (const HPair& q : P) s.push_back({((u64)q.i << 32) | q.j, q.lcm});
    std::sort(s.begin(), s.end());
    return s;
}

static bool select_min(std::vector<HPair>& P, u32& d, size_t& k) {
    d = 255;
    for (const HPair& q : P) d = std::min(d, (u32)(q.lcm >> 56));
    std::vector<HPair> rest;
    k = 0;
    for (const HPair& q : P)
        if ((u32)(q.lcm >> 56) == d)
            ++k;
        else
            rest.push_back(q);
    P.swap(rest);
    return true;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    std::ifstream in(argv[1]);
    u32 n;
    in >> n;
    std::string line;
    std::getline(in, line);
    MonoOps mo;
    mo.init(n);
    std::vector<u64> lm1, lm2, lm3;
    std::vector<u8> act1, act2, act3;
    std::vector<HPair> P1, P2, P3;
    GmScratch X, X3;
    u32 pending = 0;  // elements of the current step not yet given to state 3
    auto flush3 = [&]() {
        const u32 h1 = (u32)lm1.size(), h0 = h1 - pending;
        for (u32 h = h0; h < h1; ++h) {
            lm3.push_back(lm1[h]);
            act3.push_back(0);
        }
        gm_insert_step(mo, X3, lm3, act3, P3, h0, h1);
        pending = 0;
        return as_set(P3) == as_set(P1) && act3 == act1;
    };
    size_t ins = 0, steps = 0;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        char kind;
        if (!(ss >> kind)) continue;
        if (kind == 'S') {
            u32 d, nsel, d1, d2, d3;
            size_t k1, k2, k3;
            ss >> d >> nsel;
            if (!flush3()) {
                printf("FAIL step %zu: the step-batched insertion differs\n", steps);
                return 1;
            }
            select_min(P1, d1, k1);
            select_min(P2, d2, k2);
            select_min(P3, d3, k3);
            if (k3 != k1 || d3 != d1) {
                printf("FAIL step %zu: step-batched selection %zu/%u\n", steps, k3, d3);
                return 1;
            }
            if (d1 != d || k1 != nsel || d2 != d || k2 != nsel) {
                printf("FAIL step %zu: expected %u pairs of degree %u, generic %zu/%u, fast %zu/%u\n", steps, nsel, d,
                       k1, d1, k2, d2);
                return 1;
            }
            ++steps;
        } else {
            u64 P = 0;
            u32 deg = 0;
            for (u32 i = 0; i < n; ++i) {
                u32 a;
                ss >> a;
                P |= (u64)a << (mo.w * i);
                deg += a;
            }
            P |= (u64)deg << 56;
            const u32 h = (u32)lm1.size();
            lm1.push_back(P);
            lm2.push_back(P);
            act1.push_back(0);
            act2.push_back(0);
            gm_update(mo, lm1, act1, P1, h);
            gm_insert(mo, X, lm2, act2, P2, h);
            if (as_set(P1) != as_set(P2) || act1 != act2) {
                printf("FAIL insertion %zu: generic %zu pairs, fast %zu pairs\n", ins, P1.size(), P2.size());
                return 1;
            }
            ++ins;
            ++pending;
        }
    }
    if (!flush3()) {
        printf("FAIL final: the step-batched insertion differs\n");
        return 1;
    }
    printf("OK %zu insertions %zu steps generic=%d\n", ins, steps, (int)X.generic);
    return 0;
}
