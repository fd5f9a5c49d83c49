// Host construction of the wave-core layouts (wave.h).
#include "wave.h"

#include <algorithm>
#include <utility>

namespace gltrsv {

void build_wave_layout(const CsrView &A, bool upper, const int32_t *core, const int32_t *superstep, int32_t S,
                       const std::vector<int32_t> &perm, int64_t W, WaveLayout *out)
{
    WaveLayout &L = *out;
    const int64_t n = A.n;
    const size_t un = static_cast<size_t>(n);
    // tasks: maximal runs of equal (superstep, core) in the order, those of
    // a superstep longest first
    std::vector<std::pair<int64_t, int64_t>> tasks;   // (first position in perm, length)
    L.wsuper.assign(size_t(S) + 1, 0);
    int64_t pos = 0;
    for (int32_t s = 0; s < S; s++) {
        const size_t first = tasks.size();
        while (pos < n && superstep[perm[size_t(pos)]] == s) {
            const int32_t c = core[perm[size_t(pos)]];
            int64_t q = pos;
            while (q < n && superstep[perm[size_t(q)]] == s && core[perm[size_t(q)]] == c) q++;
            tasks.emplace_back(pos, q - pos);
            pos = q;
        }
        std::stable_sort(tasks.begin() + std::ptrdiff_t(first), tasks.end(),
                         [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
                             return a.second > b.second;
                         });
        L.wsuper[size_t(s) + 1] = int32_t(tasks.size());
    }
    // new position of every row, and the task of every new position
    L.wrow.assign(un, 0);
    std::vector<int32_t> task_of(un);
    std::vector<int64_t> newpos(un);
    L.wtask.assign(tasks.size() + 1, 0);
    int64_t np = 0;
    for (size_t t = 0; t < tasks.size(); t++) {
        L.wtask[t] = np;
        for (int64_t q = 0; q < tasks[t].second; q++, np++) {
            const int32_t v = perm[size_t(tasks[t].first + q)];
            const int32_t row = upper ? int32_t(n - 1 - v) : v;
            L.wrow[size_t(np)] = row;
            task_of[size_t(np)] = int32_t(t);
            newpos[size_t(row)] = np;
        }
    }
    L.wtask[tasks.size()] = np;
    const size_t uoff = static_cast<size_t>(std::max<int64_t>(A.nnz - n, 0));
    L.wptr.assign(un + 1, 0);
    L.wdiag.assign(un, 0.0);
    L.wcol.assign(uoff, 0u);
    L.wval.assign(uoff, 0.0);
    int64_t e = 0;
    for (int64_t t = 0; t < n; t++) {
        const int32_t row = L.wrow[size_t(t)];
        const int64_t beg = A.row_ptr[row], end = A.row_ptr[row + 1];
        L.wdiag[size_t(t)] = A.val[upper ? beg : end - 1];
        L.wptr[size_t(t)] = e;
        for (int64_t k = upper ? beg + 1 : beg; k < (upper ? end : end - 1); k++, e++) {
            const int32_t c = A.col[k];
            const int64_t pc = newpos[size_t(c)];
            const int64_t back = t - pc;
            const bool same = task_of[size_t(pc)] == task_of[size_t(t)] && back > 0 && back < kWaveRing;
            L.wcol[size_t(e)] = same ? (kIntBit | uint32_t(back)) : uint32_t(c);
            L.wval[size_t(e)] = A.val[k];
        }
    }
    L.wptr[un] = e;
    // per-wave record streams
    const int64_t T = int64_t(tasks.size());
    L.waves = W;
    L.sbeg.assign(size_t(W) + 1, 0);
    L.stask.assign(size_t(T), 0);
    L.ssize.assign(size_t(T), 0);
    int64_t so = 0;
    for (int64_t v = 0; v < W; v++) {
        L.sbeg[size_t(v)] = so;
        for (int64_t t = v; t < T; t += W) {
            L.stask[size_t(t)] = so;
            const int64_t q0 = L.wtask[size_t(t)], q1 = L.wtask[size_t(t) + 1];
            L.ssize[size_t(t)] = (q1 - q0) + (L.wptr[size_t(q1)] - L.wptr[size_t(q0)]);
            so += L.ssize[size_t(t)];
        }
        so++;   // the slot's PAD
    }
    L.sbeg[size_t(W)] = so;
    L.scol.assign(size_t(so + kStreamPad), kPadWord);
    L.sval.assign(size_t(so + kStreamPad), 0.0);
    for (int64_t t = 0; t < T; t++) {
        int64_t o = L.stask[size_t(t)];
        for (int64_t q = L.wtask[size_t(t)]; q < L.wtask[size_t(t) + 1]; q++) {
            L.scol[size_t(o)] = kHdrBit | (q == L.wtask[size_t(t)] ? kIntBit : 0u) | uint32_t(L.wrow[size_t(q)]);
            L.sval[size_t(o)] = L.wdiag[size_t(q)];
            o++;
            for (int64_t k = L.wptr[size_t(q)]; k < L.wptr[size_t(q) + 1]; k++, o++) {
                L.scol[size_t(o)] = L.wcol[size_t(k)];
                L.sval[size_t(o)] = L.wval[size_t(k)];
            }
        }
    }
}

}  // namespace gltrsv
