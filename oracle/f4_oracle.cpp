// Oracle O1: a plain, slow, textbook F4 over F_p (test infrastructure only).
//
// This file is the CPU reference that the GPU library is checked against. It
// shares no code with the GPU path: monomials are explicit exponent vectors,
// the term order is the textbook grevlex comparison, the dictionary is a
// std::map, and arithmetic is plain `% p` on 64-bit integers. Only the test
// suite, the smoke check and the benchmark's CPU-baseline leg may call it.
//
// What it computes (paper references are by section / definition / equation):
//  * S-polynomial pairs and their two "halves" (Definition "S-polynomial").
//  * One F4 step = symbolic preprocessing SP: B -> (T, R, Pi) (Definition
//    "Symbolic preprocessing operator"), with the one-step reduction closure of
//    Remark "Truncation and why symbolic preprocessing matters" and Definition
//    "Support-closure for correctness"; the Macaulay matrix of Definition
//    "Sparse Macaulay matrix for a batch", columns in descending term order.
//  * Elimination: Faugere-Lachartre split of the pivot / non-pivot columns,
//    reduction of the non-pivot rows by the pivot rows, then the reduced row
//    echelon form of the trailing block (the two-panel instance of the PSGE
//    section "PSGE: panel-structured Gaussian elimination").
//  * The full loop: Gebauer-Moeller pair update, normal selection strategy,
//    new basis elements from the echelon rows, final inter-reduction.
// Conventions where the paper is silent (reducer choice, row order, pivot row
// choice, echelon form) are fixed in the design notes and repeated at each use.
//
// C API at the bottom (extern "C"), consumed by oracle/__init__.py via ctypes.

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <utility>
#include <vector>

namespace {

typedef uint64_t u64;
typedef uint32_t u32;

// ---------------------------------------------------------------- monomials
struct Mono {
    std::vector<int> e;  // exponents a_1..a_n
    int deg = 0;
};

int g_n = 0;  // number of variables of the running system

Mono mono_from(const std::vector<int>& e) {
    Mono m;
    m.e = e;
    m.deg = 0;
    for (int a : e) m.deg += a;
    return m;
}

// grevlex with x_1 > ... > x_n: higher total degree wins; on equal degree the
// monomial whose exponent vector is smaller at the last position where the two
// differ is the larger one.  Returns +1 if a > b, -1 if a < b, 0 if equal.
int cmp(const Mono& a, const Mono& b) {
    if (a.deg != b.deg) return a.deg > b.deg ? 1 : -1;
    for (int i = g_n - 1; i >= 0; --i)
        if (a.e[i] != b.e[i]) return a.e[i] < b.e[i] ? 1 : -1;
    return 0;
}

struct Desc {  // strict "a before b" for containers sorted largest first
    bool operator()(const Mono& a, const Mono& b) const { return cmp(a, b) > 0; }
};

Mono mul(const Mono& a, const Mono& b) {
    Mono m;
    m.e.resize(g_n);
    for (int i = 0; i < g_n; ++i) m.e[i] = a.e[i] + b.e[i];
    m.deg = a.deg + b.deg;
    return m;
}

bool divides(const Mono& a, const Mono& b) {  // a | b
    for (int i = 0; i < g_n; ++i)
        if (a.e[i] > b.e[i]) return false;
    return true;
}

Mono quot(const Mono& b, const Mono& a) {  // b / a, requires a | b
    Mono m;
    m.e.resize(g_n);
    for (int i = 0; i < g_n; ++i) m.e[i] = b.e[i] - a.e[i];
    m.deg = b.deg - a.deg;
    return m;
}

Mono lcm(const Mono& a, const Mono& b) {
    Mono m;
    m.e.resize(g_n);
    m.deg = 0;
    for (int i = 0; i < g_n; ++i) {
        m.e[i] = std::max(a.e[i], b.e[i]);
        m.deg += m.e[i];
    }
    return m;
}

bool coprime(const Mono& a, const Mono& b) {
    for (int i = 0; i < g_n; ++i)
        if (a.e[i] > 0 && b.e[i] > 0) return false;
    return true;
}

bool equal(const Mono& a, const Mono& b) { return cmp(a, b) == 0; }

// --------------------------------------------------------------- arithmetic
u64 g_p = 0;

u64 addm(u64 a, u64 b) { return (a + b) % g_p; }
u64 subm(u64 a, u64 b) { return (a + g_p - b) % g_p; }
u64 mulm(u64 a, u64 b) { return (a * b) % g_p; }  // a, b < 2^31, product < 2^62
u64 powm(u64 a, u64 e) {
    u64 r = 1 % g_p;
    a %= g_p;
    while (e) {
        if (e & 1) r = mulm(r, a);
        a = mulm(a, a);
        e >>= 1;
    }
    return r;
}
u64 invm(u64 a) { return powm(a, g_p - 2); }  // Fermat: a^(p-2) = a^-1 for prime p

// ------------------------------------------------------------- polynomials
struct Term {
    Mono m;
    u64 c;
};
typedef std::vector<Term> Poly;  // sorted by monomial, largest first; no zero coefficients

const Mono& LM(const Poly& f) { return f[0].m; }

Poly monic(const Poly& f) {
    Poly g = f;
    if (g.empty()) return g;
    u64 inv = invm(g[0].c);
    for (auto& t : g) t.c = mulm(t.c, inv);
    return g;
}

// f - c * s * h  (plain merge of two sorted term lists)
Poly sub_scaled(const Poly& f, u64 c, const Mono& s, const Poly& h) {
    Poly out;
    size_t i = 0, j = 0;
    while (i < f.size() || j < h.size()) {
        if (j == h.size()) {
            out.push_back(f[i++]);
            continue;
        }
        Mono hm = mul(s, h[j].m);
        u64 hv = mulm(c, h[j].c);
        int k = (i == f.size()) ? -1 : cmp(f[i].m, hm);
        if (k > 0) {
            out.push_back(f[i++]);
        } else if (k < 0) {
            out.push_back({hm, subm(0, hv)});
            ++j;
        } else {
            u64 v = subm(f[i].c, hv);
            if (v) out.push_back({hm, v});
            ++i;
            ++j;
        }
    }
    return out;
}

// ------------------------------------------------------------------- state
struct Pair {
    int i, j;  // basis indices, i < j
    Mono lcm;
};

struct Recorded {
    std::map<std::string, std::vector<u64>> arrays;
};

struct Oracle {
    int n = 0;
    u64 p = 0;
    std::vector<Poly> input;
    std::vector<Poly> G;
    std::vector<char> active;
    std::vector<Pair> P;
    std::map<std::string, std::vector<u64>> out;  // named result arrays
    int record = -1;                              // -1 none, -2 all, k >= 0 only step k
    int stop_after = -1;                          // -1 run to completion
    int stop_deg = -1;                            // stop after the first step of this degree
    bool unit = false;                            // basis became {1}
};

void push_mono(std::vector<u64>& v, const Mono& m) {
    for (int i = 0; i < g_n; ++i) v.push_back((u64)m.e[i]);
}

// Gebauer-Moeller update (Becker-Weispfenning form) inserting h = G[hidx].
void gm_update(Oracle& S, int hidx) {
    const Mono& lh = LM(S.G[hidx]);
    // C: pairs (h, g) for active g, ascending g
    std::vector<int> C;
    for (int g = 0; g < hidx; ++g)
        if (S.active[g]) C.push_back(g);
    std::vector<Mono> Clcm;
    for (int g : C) Clcm.push_back(lcm(lh, LM(S.G[g])));
    std::vector<char> inC(C.size(), 1), inD(C.size(), 0);
    for (size_t a = 0; a < C.size(); ++a) {
        inC[a] = 0;
        bool keep = coprime(lh, LM(S.G[C[a]]));
        if (!keep) {
            bool covered = false;
            for (size_t b = 0; b < C.size() && !covered; ++b)
                if (b != a && (inC[b] || inD[b]) && divides(Clcm[b], Clcm[a])) covered = true;
            keep = !covered;
        }
        if (keep) inD[a] = 1;
    }
    // E: kept pairs minus those with coprime leading monomials (product criterion)
    std::vector<Pair> E;
    for (size_t a = 0; a < C.size(); ++a)
        if (inD[a] && !coprime(lh, LM(S.G[C[a]]))) E.push_back({C[a], hidx, Clcm[a]});
    // prune old pairs (chain criterion)
    std::vector<Pair> Pn;
    for (const Pair& q : S.P) {
        bool drop = divides(lh, q.lcm) && !equal(lcm(LM(S.G[q.i]), lh), q.lcm) &&
                    !equal(lcm(lh, LM(S.G[q.j])), q.lcm);
        if (!drop) Pn.push_back(q);
    }
    for (const Pair& q : E) Pn.push_back(q);
    S.P.swap(Pn);
    // deactivate elements whose leading monomial is a multiple of LM(h)
    for (int g = 0; g < hidx; ++g)
        if (S.active[g] && divides(lh, LM(S.G[g]))) S.active[g] = 0;
    S.active[hidx] = 1;
}

void insert_basis(Oracle& S, const Poly& h) {
    S.G.push_back(h);
    S.active.push_back(0);
    gm_update(S, (int)S.G.size() - 1);
}

struct Row {
    Mono t;
    int k;
    Mono lm;
};

double now_ns() {
    return (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// One F4 step on the selected pairs.  Returns the new basis elements (monic,
// largest leading monomial first).
std::vector<Poly> f4_step(Oracle& S, int step, const std::vector<Pair>& sel, int d) {
    bool rec = (S.record == -2 || S.record == step);
    std::string pre = "s" + std::to_string(step) + ".";
    double t0 = now_ns();

    if (rec) {  // snapshot of the basis and the selection the step starts from
        std::vector<u64> gp{0}, ge, gc, ga;
        for (size_t k = 0; k < S.G.size(); ++k) {
            for (const Term& t : S.G[k]) {
                push_mono(ge, t.m);
                gc.push_back(t.c);
            }
            gp.push_back(gc.size());
            ga.push_back((u64)S.active[k]);
        }
        S.out[pre + "G.ptr"] = gp;
        S.out[pre + "G.exp"] = ge;
        S.out[pre + "G.coeff"] = gc;
        S.out[pre + "G.active"] = ga;
        std::vector<u64> sv;
        for (const Pair& q : sel) {
            sv.push_back((u64)q.i);
            sv.push_back((u64)q.j);
        }
        S.out[pre + "sel"] = sv;
    }

    // --- halves: (lcm / LM(g_i), i) and (lcm / LM(g_j), j), duplicates collapse
    auto row_less = [](const Row& a, const Row& b) {  // identity order on (t, k)
        if (a.k != b.k) return a.k < b.k;
        return cmp(a.t, b.t) > 0;
    };
    std::set<Row, decltype(row_less)> rowset(row_less);
    for (const Pair& q : sel) {
        rowset.insert({quot(q.lcm, LM(S.G[q.i])), q.i, q.lcm});
        rowset.insert({quot(q.lcm, LM(S.G[q.j])), q.j, q.lcm});
    }
    std::vector<Row> rows(rowset.begin(), rowset.end());

    // --- symbolic preprocessing: T = union of supports, closed under one-step
    // reduction by the most recently inserted active divisor.
    std::set<Mono, Desc> T, Done;
    std::vector<Mono> work;
    auto add_support = [&](const Row& rw) {
        for (const Term& t : S.G[rw.k]) {
            Mono u = mul(rw.t, t.m);
            if (T.insert(u).second) work.push_back(u);
        }
    };
    for (const Row& rw : rows) Done.insert(rw.lm);
    for (const Row& rw : rows) add_support(rw);
    while (!work.empty()) {
        Mono m = work.back();
        work.pop_back();
        if (Done.count(m)) continue;
        Done.insert(m);
        int best = -1;
        for (int g = (int)S.G.size() - 1; g >= 0; --g)
            if (S.active[g] && divides(LM(S.G[g]), m)) {
                best = g;
                break;
            }
        if (best >= 0) {
            Row rw{quot(m, LM(S.G[best])), best, m};
            rows.push_back(rw);
            add_support(rw);
        }
    }

    // --- row order: leading monomial descending, then basis index ascending,
    // then shift descending.
    std::sort(rows.begin(), rows.end(), [](const Row& a, const Row& b) {
        int c = cmp(a.lm, b.lm);
        if (c != 0) return c > 0;
        if (a.k != b.k) return a.k < b.k;
        return cmp(a.t, b.t) > 0;
    });

    // --- columns: T in descending order, index 0 = largest monomial
    std::vector<Mono> cols(T.begin(), T.end());
    std::map<std::vector<int>, u32> colidx;
    for (size_t c = 0; c < cols.size(); ++c) colidx[cols[c].e] = (u32)c;
    const size_t N = cols.size(), r = rows.size();

    // --- CSR of A: row i = coefficients of t_i * g_{k_i} on the columns
    std::vector<u32> row_ptr{0}, col_ind, val;
    for (const Row& rw : rows) {
        for (const Term& t : S.G[rw.k]) {
            col_ind.push_back(colidx.at(mul(rw.t, t.m).e));
            val.push_back((u32)t.c);
        }
        row_ptr.push_back((u32)col_ind.size());
    }
    double t1 = now_ns();

    // --- elimination.  Pivot columns: the leading column of every row.
    std::vector<int> pivrow(N, -1);
    for (size_t i = 0; i < r; ++i) {
        u32 lead = col_ind[row_ptr[i]];
        u32 len = row_ptr[i + 1] - row_ptr[i];
        int cur = pivrow[lead];
        if (cur < 0 || len < row_ptr[cur + 1] - row_ptr[cur]) pivrow[lead] = (int)i;
    }
    std::vector<char> is_pivot_row(r, 0);
    size_t npiv = 0;
    for (size_t c = 0; c < N; ++c)
        if (pivrow[c] >= 0) {
            is_pivot_row[pivrow[c]] = 1;
            ++npiv;
        }
    // monic copies of the pivot rows, as (col, val) lists
    std::vector<std::vector<std::pair<u32, u64>>> U(N);
    for (size_t c = 0; c < N; ++c) {
        if (pivrow[c] < 0) continue;
        int i = pivrow[c];
        u64 inv = invm(val[row_ptr[i]]);
        for (u32 q = row_ptr[i]; q < row_ptr[i + 1]; ++q) U[c].push_back({col_ind[q], mulm(val[q], inv)});
    }
    // reduce every non-pivot row by the pivot rows, left to right
    std::vector<std::vector<u64>> Dp;  // trailing block rows (dense over all N columns)
    for (size_t i = 0; i < r; ++i) {
        if (is_pivot_row[i]) continue;
        std::vector<u64> acc(N, 0);
        for (u32 q = row_ptr[i]; q < row_ptr[i + 1]; ++q) acc[col_ind[q]] = val[q];
        for (size_t c = 0; c < N; ++c) {
            if (acc[c] == 0 || pivrow[c] < 0) continue;
            u64 f = acc[c];
            for (const auto& e : U[c]) acc[e.first] = subm(acc[e.first], mulm(f, e.second));
        }
        Dp.push_back(acc);
    }
    // reduced row echelon form of the trailing block (non-pivot columns only)
    std::vector<size_t> rref_rows;  // indices into Dp, in pivot-column order
    std::vector<u32> rref_cols;
    std::vector<char> used(Dp.size(), 0);
    for (size_t c = 0; c < N; ++c) {
        if (pivrow[c] >= 0) continue;
        size_t pr = Dp.size();
        for (size_t i = 0; i < Dp.size(); ++i)
            if (!used[i] && Dp[i][c] != 0) {
                pr = i;
                break;
            }
        if (pr == Dp.size()) continue;
        used[pr] = 1;
        u64 inv = invm(Dp[pr][c]);
        for (size_t q = 0; q < N; ++q) Dp[pr][q] = mulm(Dp[pr][q], inv);
        for (size_t i = 0; i < Dp.size(); ++i) {
            if (i == pr || Dp[i][c] == 0) continue;
            u64 f = Dp[i][c];
            for (size_t q = 0; q < N; ++q)
                if (Dp[pr][q]) Dp[i][q] = subm(Dp[i][q], mulm(f, Dp[pr][q]));
        }
        rref_rows.push_back(pr);
        rref_cols.push_back((u32)c);
    }
    double t2 = now_ns();

    std::vector<Poly> news;
    std::vector<u32> rp{0}, rc, rv;
    for (size_t a = 0; a < rref_rows.size(); ++a) {
        const std::vector<u64>& row = Dp[rref_rows[a]];
        Poly h;
        for (size_t q = 0; q < N; ++q)
            if (row[q]) {
                h.push_back({cols[q], row[q]});
                rc.push_back((u32)q);
                rv.push_back((u32)row[q]);
            }
        rp.push_back((u32)rc.size());
        news.push_back(h);
    }

    const size_t rho = rref_rows.size();
    for (u64 v : {(u64)d, (u64)r, (u64)N, (u64)col_ind.size(), (u64)npiv, (u64)(npiv + rho), (u64)rho})
        S.out["steps"].push_back(v);
    S.out["time"].push_back((u64)(t1 - t0));
    S.out["time"].push_back((u64)(t2 - t1));

    if (rec) {
        std::vector<u64> v;
        auto put32 = [&](const char* name, const std::vector<u32>& a) {
            S.out[pre + name] = std::vector<u64>(a.begin(), a.end());
        };
        put32("row_ptr", row_ptr);
        put32("col_ind", col_ind);
        put32("val", val);
        std::vector<u64> te;
        for (const Mono& m : cols) push_mono(te, m);
        S.out[pre + "T"] = te;
        std::vector<u64> rt, rk;
        for (const Row& rw : rows) {
            push_mono(rt, rw.t);
            rk.push_back((u64)rw.k);
        }
        S.out[pre + "rows.t"] = rt;
        S.out[pre + "rows.k"] = rk;
        std::vector<u64> pc, pr;
        for (size_t c = 0; c < N; ++c)
            if (pivrow[c] >= 0) {
                pc.push_back(c);
                pr.push_back((u64)pivrow[c]);
            }
        S.out[pre + "pivot_cols"] = pc;
        S.out[pre + "pivot_rows"] = pr;
        put32("rref_ptr", rp);
        put32("rref_col", rc);
        put32("rref_val", rv);
        S.out[pre + "d"] = {(u64)d};
    }
    return news;
}

// Normal form of f with respect to the list H (textbook multivariate division).
Poly normal_form(const Poly& f, const std::vector<const Poly*>& H) {
    Poly rem, cur = f;
    while (!cur.empty()) {
        const Poly* red = nullptr;
        for (const Poly* h : H)
            if (divides(LM(*h), cur[0].m)) {
                red = h;
                break;
            }
        if (red) {
            u64 c = mulm(cur[0].c, invm((*red)[0].c));
            cur = sub_scaled(cur, c, quot(cur[0].m, LM(*red)), *red);
        } else {
            rem.push_back(cur[0]);
            cur.erase(cur.begin());
        }
    }
    return rem;
}

void store_basis(Oracle& S, const std::vector<Poly>& B) {
    std::vector<u64> gp{0}, ge, gc;
    for (const Poly& f : B) {
        for (const Term& t : f) {
            push_mono(ge, t.m);
            gc.push_back(t.c);
        }
        gp.push_back(gc.size());
    }
    S.out["gb.ptr"] = gp;
    S.out["gb.exp"] = ge;
    S.out["gb.coeff"] = gc;
}

int run(Oracle& S) {
    g_n = S.n;
    g_p = S.p;
    S.G.clear();
    S.active.clear();
    S.P.clear();
    S.out.clear();
    S.out["steps"] = {};
    S.out["time"] = {};
    S.unit = false;
    Mono one = mono_from(std::vector<int>(S.n, 0));
    // 1. monic inputs, zeros dropped; a nonzero constant means the unit ideal
    for (const Poly& f : S.input) {
        if (f.empty()) continue;
        Poly h = monic(f);
        if (LM(h).deg == 0) S.unit = true;
        if (!S.unit) insert_basis(S, h);
    }
    // 2. main loop
    int step = 0;
    while (!S.unit && !S.P.empty()) {
        if (S.stop_after >= 0 && step > S.stop_after) break;
        int d = S.P[0].lcm.deg;
        for (const Pair& q : S.P) d = std::min(d, q.lcm.deg);
        std::vector<Pair> sel, rest;
        for (const Pair& q : S.P) (q.lcm.deg == d ? sel : rest).push_back(q);
        S.P.swap(rest);
        std::vector<Poly> news = f4_step(S, step, sel, d);
        ++step;
        if (S.stop_deg >= 0 && d == S.stop_deg) {
            S.out["nsteps"] = {(u64)step};
            S.out["complete"] = {0};
            return 0;
        }
        for (const Poly& h : news) {
            if (LM(h).deg == 0) {
                S.unit = true;
                break;
            }
            insert_basis(S, h);
        }
    }
    S.out["nsteps"] = {(u64)step};
    if (S.stop_after >= 0 && step > S.stop_after && !S.unit && !S.P.empty()) {
        S.out["complete"] = {0};
        return 0;
    }
    S.out["complete"] = {1};
    // 3. reduced basis: minimal leading monomials, tails reduced, monic, sorted
    std::vector<Poly> B;
    if (S.unit) {
        B.push_back(Poly{{one, 1}});
    } else {
        std::vector<int> keep;
        for (size_t g = 0; g < S.G.size(); ++g) {
            if (!S.active[g]) continue;
            bool minimal = true;
            for (size_t h = 0; h < S.G.size() && minimal; ++h)
                if (h != g && S.active[h] && divides(LM(S.G[h]), LM(S.G[g]))) minimal = false;
            if (minimal) keep.push_back((int)g);
        }
        for (int g : keep) {
            std::vector<const Poly*> H;
            for (int h : keep)
                if (h != g) H.push_back(&S.G[h]);
            Poly tail(S.G[g].begin() + 1, S.G[g].end());
            Poly red = normal_form(tail, H);
            Poly f{S.G[g][0]};
            f.insert(f.end(), red.begin(), red.end());
            B.push_back(monic(f));
        }
        std::sort(B.begin(), B.end(), [](const Poly& a, const Poly& b) { return cmp(LM(a), LM(b)) > 0; });
    }
    store_basis(S, B);
    return 0;
}

}  // namespace

extern "C" {

void* or_create(uint32_t n, uint32_t p) {
    if (n == 0 || n > 64 || p < 3) return nullptr;
    Oracle* S = new Oracle();
    S->n = (int)n;
    S->p = p;
    return S;
}

void or_destroy(void* h) { delete (Oracle*)h; }

// Add one input polynomial: nterms terms, exps row-major (nterms x n), integer
// coefficients reduced mod p here; repeated monomials are summed.
int or_add_poly(void* h, uint32_t nterms, const uint32_t* exps, const uint64_t* coeffs) {
    Oracle& S = *(Oracle*)h;
    g_n = S.n;
    g_p = S.p;
    std::map<Mono, u64, Desc> acc;
    for (uint32_t t = 0; t < nterms; ++t) {
        std::vector<int> e(S.n);
        for (int i = 0; i < S.n; ++i) {
            if (exps[(size_t)t * S.n + i] > 200) return 1;
            e[i] = (int)exps[(size_t)t * S.n + i];
        }
        Mono m = mono_from(e);
        acc[m] = addm(acc[m], coeffs[t] % S.p);
    }
    Poly f;
    for (auto& kv : acc)
        if (kv.second) f.push_back({kv.first, kv.second});
    S.input.push_back(f);
    return 0;
}

void or_set_record(void* h, int32_t step) { ((Oracle*)h)->record = step; }
void or_set_stop(void* h, int32_t step) { ((Oracle*)h)->stop_after = step; }
void or_set_stop_deg(void* h, int32_t deg) { ((Oracle*)h)->stop_deg = deg; }
int or_run(void* h) { return run(*(Oracle*)h); }

int64_t or_len(void* h, const char* name) {
    Oracle& S = *(Oracle*)h;
    auto it = S.out.find(name);
    return it == S.out.end() ? -1 : (int64_t)it->second.size();
}

int or_get(void* h, const char* name, uint64_t* dst) {
    Oracle& S = *(Oracle*)h;
    auto it = S.out.find(name);
    if (it == S.out.end()) return 1;
    if (!it->second.empty()) std::memcpy(dst, it->second.data(), it->second.size() * sizeof(u64));
    return 0;
}

}  // extern "C"
