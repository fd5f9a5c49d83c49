// Test driver for the host analysis under AddressSanitizer,
// UndefinedBehaviorSanitizer and ThreadSanitizer (built by
// tests/test_sanitize.py with g++; no GPU code is involved).
//
// Input file: int64 n, int64 nnz, int32 upper, int64 row_ptr[n+1],
// int32 col[nnz], double val[nnz].  For a lower-triangular matrix the driver
// runs every scheduler of the library (GrowLocal, Algorithm 3.1, with one and
// several workers; block-parallel, Sec. 3.1; Funnel + GrowLocal, Sec. 4; the
// wavefront schedule), checks each against Definition 2.1, orders (Sec. 5)
// and packs it, and feeds malformed copies of the matrix to the CSR check.
// For an upper-triangular one it runs the mirrored path of backward
// substitution.  The GrowLocal schedule of the first parameter set is written
// to the output file (int32 core[n], int32 superstep[n]) for comparison with
// the oracle.  Exit status 0 = every check passed.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "analysis.h"

using namespace gltrsv;

namespace {

int fails = 0;

void expect(bool ok, const char *what, const std::string &msg = "")
{
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s %s\n", what, msg.c_str());
        fails++;
    }
}

template <class T>
bool read_all(std::FILE *f, std::vector<T> &v, size_t count)
{
    v.resize(count);
    return count == 0 || std::fread(v.data(), sizeof(T), count, f) == count;
}

// Orders, lays out and fills the stream of a schedule, and checks that the
// one-pass pack agrees with the two-phase layout + fill.
void pack_and_check(const CsrView &D, const CsrView &V, const Schedule &s, bool upper, const char *label)
{
    std::string msg;
    expect(validate_schedule(D, s, &msg) == 0, label, msg);
    std::vector<int32_t> perm = schedule_order(D.n, s.core.data(), s.superstep.data(), s.S);
    expect(int64_t(perm.size()) == D.n, label, "order size");
    std::vector<char> seen(size_t(D.n), 0);
    for (int32_t r : perm) {
        expect(r >= 0 && r < D.n && !seen[size_t(r)], label, "order is not a permutation");
        if (r >= 0 && r < D.n) seen[size_t(r)] = 1;
    }
    PackLayout lay = pack_layout(D, s, perm);
    if (upper) {
        pack_fill_upper(V, perm, lay);
    } else {
        pack_fill(V, s, perm, lay);
        Packed one = pack_stream(V, s, perm);
        expect(one.word == lay.pk.word && one.value == lay.pk.value, label, "pack_stream differs from layout + fill");
    }
    expect(lay.pk.slots >= D.nnz, label, "fewer slots than entries");
    const CostModel cm;
    const double a = predict_cost_us(D, s, perm, cm), b = predict_async_us(D, s, perm, cm);
    expect(a >= 0.0 && b >= 0.0, label, "negative prediction");
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc < 3) {
        std::fprintf(stderr, "usage: %s matrix.bin schedule.out [threads]\n", argv[0]);
        return 2;
    }
    const int32_t threads = argc > 3 ? std::atoi(argv[3]) : 4;
    std::FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n = 0, nnz = 0;
    int32_t upper = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<double> val;
    bool ok = std::fread(&n, 8, 1, f) == 1 && std::fread(&nnz, 8, 1, f) == 1 && std::fread(&upper, 4, 1, f) == 1;
    ok = ok && read_all(f, rp, size_t(n + 1)) && read_all(f, col, size_t(nnz)) && read_all(f, val, size_t(nnz));
    std::fclose(f);
    if (!ok) return 2;

    CsrView V;
    V.n = n;
    V.nnz = nnz;
    V.row_ptr = rp.data();
    V.col = col.data();
    V.val = val.data();
    std::string msg;
    expect((upper ? check_csr_upper(V, true, &msg) : check_csr(V, true, &msg)) == 0, "csr check", msg);
    Mirror mir;
    if (upper) mir = mirror_upper(V);
    const CsrView D = upper ? mir.view() : V;

    struct Case {
        const char *label;
        SchedParams p;
    };
    std::vector<Case> cases;
    SchedParams base;
    base.k = 4;
    base.L = 10.0;
    base.alpha0 = 1.0;
    base.threads = 1;
    cases.push_back({"growlocal k=4 one worker", base});
    SchedParams p = base;
    p.threads = threads;
    cases.push_back({"growlocal k=4 worker pool", p});
    p = SchedParams();
    p.threads = threads;
    cases.push_back({"growlocal paper parameters", p});
    p = base;
    p.k = 65536;
    p.L = 50.0;
    p.threads = threads;
    cases.push_back({"growlocal k=65536", p});
    p = base;
    p.k = 64;
    p.blocks = 3;
    p.threads = threads;
    cases.push_back({"block-parallel, 3 blocks", p});
    p = base;
    p.k = 8;
    p.funnel_max_weight = 16;
    cases.push_back({"funnel cap 16", p});

    std::vector<int32_t> lv;
    const int32_t levels = wavefront_levels(D, lv);
    expect(n == 0 || levels >= 1, "wavefront levels");
    Schedule w = schedule_wavefront(D);
    expect(w.S == levels, "wavefront supersteps");
    pack_and_check(D, V, w, upper != 0, "wavefront");

    Schedule first;
    for (size_t c = 0; c < cases.size(); c++) {
        Schedule s = schedule_growlocal(D, cases[c].p);
        expect(s.S <= levels || n == 0, cases[c].label, "more supersteps than wavefronts");
        pack_and_check(D, V, s, upper != 0, cases[c].label);
        if (c == 0) first = s;
    }
    if (!upper) {
        const ReducedDag r = transitive_reduction(D);
        int32_t parts = 0;
        const std::vector<int32_t> part = funnel_partition(D, r, 8, &parts);
        for (int32_t q : part) expect(q >= 0 && q < parts, "funnel part index");
    }
    (void)pattern_key(V);

    // malformed copies must be rejected with an error code, not crash
    if (!upper && n >= 3) {
        auto row_with = [&](int64_t len) {
            for (int64_t r = 0; r < n; r++)
                if (rp[size_t(r + 1)] - rp[size_t(r)] >= len) return r;
            return int64_t(-1);
        };
        CsrView B = V;
        const int64_t r2 = row_with(2), r3 = row_with(3);
        if (r2 >= 0) {
            const int64_t a = rp[size_t(r2)], d = rp[size_t(r2 + 1)] - 1;
            std::vector<int32_t> bad = col;
            bad[size_t(a)] = int32_t(n + 5);                     // column out of range
            B.col = bad.data();
            expect(check_csr(B, true, &msg) != 0, "out-of-range column accepted");
            bad = col;
            bad[size_t(d)] = bad[size_t(a)];                     // diagonal missing
            B.col = bad.data();
            expect(check_csr(B, true, &msg) != 0, "missing diagonal accepted");
            std::vector<double> zv = val;
            zv[size_t(d)] = 0.0;                                 // zero diagonal
            B = V;
            B.val = zv.data();
            expect(check_csr(B, true, &msg) != 0, "zero diagonal accepted");
            B = V;
        }
        if (r3 >= 0) {
            const int64_t a = rp[size_t(r3)];
            std::vector<int32_t> bad = col;
            bad[size_t(a + 1)] = bad[size_t(a)];                 // repeated column
            B.col = bad.data();
            expect(check_csr(B, true, &msg) != 0, "repeated column accepted");
            B = V;
        }
        std::vector<int64_t> brp = rp;
        brp[1] = brp[2] + 1;                                     // row pointers not monotone
        B.row_ptr = brp.data();
        expect(check_csr(B, true, &msg) != 0, "non-monotone row pointers accepted");
    }

    std::FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 2;
    std::vector<int32_t> core(static_cast<size_t>(n)), sup(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; i++) {
        const int64_t v = upper ? n - 1 - i : i;   // per row of the given matrix
        core[size_t(i)] = first.core[size_t(v)];
        sup[size_t(i)] = first.superstep[size_t(v)];
    }
    if (n > 0) {
        std::fwrite(core.data(), 4, size_t(n), o);
        std::fwrite(sup.data(), 4, size_t(n), o);
    }
    std::fclose(o);
    if (fails) return 1;
    std::printf("ok n=%lld nnz=%lld S=%d\n", (long long)n, (long long)nnz, first.S);
    return 0;
}
