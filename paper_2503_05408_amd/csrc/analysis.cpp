// Host-side analysis: CSR checks, wavefronts, GrowLocal (Algorithm 3.1),
// the schedule order of Sec. 5 and the packed layout of the device stream.
#include "analysis.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>

#include "../../include/gltrsv.h"

namespace gltrsv {

int check_csr(const CsrView &A, bool need_values, std::string *msg)
{
    auto fail = [&](int code, const std::string &m) {
        if (msg) *msg = m;
        return code;
    };
    if (A.n < 0 || A.nnz < 0) return fail(GLTRSV_EINVAL, "negative size");
    if (A.n > kMaxRows) return fail(GLTRSV_ERANGE, "n exceeds 2^30 - 1");
    if (A.n == 0) return GLTRSV_OK;
    if (!A.row_ptr || !A.col) return fail(GLTRSV_EINVAL, "null row_ptr or col");
    if (need_values && !A.val) return fail(GLTRSV_EINVAL, "null values");
    if (A.row_ptr[0] != 0 || A.row_ptr[A.n] != A.nnz)
        return fail(GLTRSV_ERANGE, "row_ptr[0] != 0 or row_ptr[n] != nnz");
    for (int64_t i = 0; i < A.n; i++) {
        const int64_t lo = A.row_ptr[i], hi = A.row_ptr[i + 1];
        if (hi < lo) return fail(GLTRSV_ERANGE, "row_ptr decreases at row " + std::to_string(i));
        if (hi == lo) return fail(GLTRSV_ESINGULAR, "row " + std::to_string(i) + " has no diagonal");
        int32_t prev = -1;
        for (int64_t e = lo; e < hi; e++) {
            const int32_t c = A.col[e];
            if (c < 0 || c >= A.n) return fail(GLTRSV_ERANGE, "column out of range in row " + std::to_string(i));
            if (c > i) return fail(GLTRSV_ENOTLOWER, "entry above the diagonal in row " + std::to_string(i));
            if (c <= prev) return fail(GLTRSV_EUNSORTED, "columns not strictly rising in row " + std::to_string(i));
            prev = c;
        }
        if (A.col[hi - 1] != i) return fail(GLTRSV_ESINGULAR, "row " + std::to_string(i) + " has no diagonal");
        if (need_values && A.val[hi - 1] == 0.0)
            return fail(GLTRSV_ESINGULAR, "zero diagonal in row " + std::to_string(i));
    }
    return GLTRSV_OK;
}

int check_csr_upper(const CsrView &A, bool need_values, std::string *msg)
{
    auto fail = [&](int code, const std::string &m) {
        if (msg) *msg = m;
        return code;
    };
    if (A.n < 0 || A.nnz < 0) return fail(GLTRSV_EINVAL, "negative size");
    if (A.n > kMaxRows) return fail(GLTRSV_ERANGE, "n exceeds 2^30 - 1");
    if (A.n == 0) return GLTRSV_OK;
    if (!A.row_ptr || !A.col) return fail(GLTRSV_EINVAL, "null row_ptr or col");
    if (need_values && !A.val) return fail(GLTRSV_EINVAL, "null values");
    if (A.row_ptr[0] != 0 || A.row_ptr[A.n] != A.nnz)
        return fail(GLTRSV_ERANGE, "row_ptr[0] != 0 or row_ptr[n] != nnz");
    for (int64_t i = 0; i < A.n; i++) {
        const int64_t lo = A.row_ptr[i], hi = A.row_ptr[i + 1];
        if (hi < lo) return fail(GLTRSV_ERANGE, "row_ptr decreases at row " + std::to_string(i));
        if (hi == lo) return fail(GLTRSV_ESINGULAR, "row " + std::to_string(i) + " has no diagonal");
        int32_t prev = -1;
        for (int64_t e = lo; e < hi; e++) {
            const int32_t c = A.col[e];
            if (c < 0 || c >= A.n) return fail(GLTRSV_ERANGE, "column out of range in row " + std::to_string(i));
            if (c < i) return fail(GLTRSV_ENOTLOWER, "entry below the diagonal in row " + std::to_string(i));
            if (c <= prev) return fail(GLTRSV_EUNSORTED, "columns not strictly rising in row " + std::to_string(i));
            prev = c;
        }
        if (A.col[lo] != i) return fail(GLTRSV_ESINGULAR, "row " + std::to_string(i) + " has no diagonal");
        if (need_values && A.val[lo] == 0.0)
            return fail(GLTRSV_ESINGULAR, "zero diagonal in row " + std::to_string(i));
    }
    return GLTRSV_OK;
}

Mirror mirror_upper(const CsrView &U)
{
    Mirror m;
    const int64_t n = U.n;
    m.row_ptr.assign(size_t(n) + 1, 0);
    m.col.resize(size_t(U.nnz));
    for (int64_t v = 0; v < n; v++) {
        const int64_t i = n - 1 - v;
        m.row_ptr[size_t(v) + 1] = m.row_ptr[size_t(v)] + (U.row_ptr[i + 1] - U.row_ptr[i]);
    }
    for (int64_t v = 0; v < n; v++) {
        const int64_t i = n - 1 - v, lo = U.row_ptr[i], hi = U.row_ptr[i + 1];
        int64_t o = m.row_ptr[size_t(v)];
        for (int64_t e = hi - 1; e > lo; e--) m.col[size_t(o++)] = int32_t(n - 1 - U.col[e]);   // rising
        m.col[size_t(o)] = int32_t(v);                                                         // diagonal
    }
    return m;
}

int32_t wavefront_levels(const CsrView &A, std::vector<int32_t> &level)
{
    level.assign(A.n, 0);
    int32_t top = 0;
    for (int64_t i = 0; i < A.n; i++) {
        int32_t best = 0;
        const int64_t last = A.row_ptr[i + 1] - 1;
        for (int64_t e = A.row_ptr[i]; e < last; e++) best = std::max(best, level[A.col[e]]);
        level[i] = best + 1;
        top = std::max(top, best + 1);
    }
    return top;
}

int validate_schedule(const CsrView &A, const Schedule &s, std::string *msg)
{
    for (int64_t i = 0; i < A.n; i++) {
        if (s.core[size_t(i)] < 0 || s.superstep[size_t(i)] < 0 || s.superstep[size_t(i)] >= s.S) {
            if (msg) *msg = "core or superstep out of range at vertex " + std::to_string(i);
            return GLTRSV_EINVAL;
        }
        for (int64_t e = A.row_ptr[i]; e < A.row_ptr[i + 1] - 1; e++) {
            const int32_t j = A.col[e];
            const bool before = s.superstep[size_t(j)] < s.superstep[size_t(i)];
            const bool same = s.superstep[size_t(j)] == s.superstep[size_t(i)] && s.core[size_t(j)] == s.core[size_t(i)];
            if (!before && !same) {
                if (msg) *msg = "edge " + std::to_string(j) + " -> " + std::to_string(i) + " violates Definition 2.1";
                return GLTRSV_EINVAL;
            }
        }
    }
    return GLTRSV_OK;
}

Schedule schedule_wavefront(const CsrView &A)
{
    Schedule s;
    std::vector<int32_t> level;
    s.S = wavefront_levels(A, level);
    s.core.resize(A.n);
    s.superstep.resize(A.n);
    std::vector<int32_t> width(s.S + 1, 0);
    for (int64_t i = 0; i < A.n; i++) {
        const int32_t lv = level[i] - 1;
        s.superstep[i] = lv;
        s.core[i] = width[lv]++;
    }
    return s;
}

// ---------------------------------------------------------------------------
// GrowLocal
// ---------------------------------------------------------------------------
namespace {

// Runs f(lo, hi) over `threads` contiguous slices of [0, n).
template <class F>
void parallel_rows(int threads, int64_t n, F f)
{
    if (threads <= 1 || n < 4096) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::thread> t;
    for (int i = 1; i < threads; i++) t.emplace_back([=] { f(n * i / threads, n * (i + 1) / threads); });
    f(int64_t(0), n / threads);
    for (std::thread &x : t) x.join();
}

// The iterations of one superstep (alpha, growth * alpha, ...) all start from
// the same barrier state, so they are independent: a pool of workers runs
// several of them at once, each with private trial state, and the acceptance
// rule then reads their results in order.  The outcome does not depend on the
// number of workers.
class GrowLocalScheduler {
public:
    // weight: vertex weights, or nullptr for the stored entries of each row
    GrowLocalScheduler(const CsrView &A, const SchedParams &p, int workers, const int64_t *weight = nullptr)
        : A_(A), p_(p)
    {
        const int64_t n = A.n;
        const int nw = std::max(1, workers);
        weight_.resize(n);
        waiting_.resize(n);
        parallel_rows(nw, n, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo; v < hi; v++) {
                const int64_t d = A.row_ptr[v + 1] - A.row_ptr[v];
                weight_[v] = weight ? weight[v] : d;   // stored entries, diagonal included
                waiting_[v] = int32_t(d - 1);         // parents = stored off-diagonals
            }
        });
        // children lists (the transpose of the strict lower part), children
        // in rising order; worker i owns the parents in its slice of [0, n)
        // and scans every row, so no two workers write the same counter
        kids_begin_.assign(n + 1, 0);
        parallel_rows(nw, n, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo + 1; v < n; v++)
                for (int64_t e = A.row_ptr[v]; e < A.row_ptr[v + 1] - 1; e++) {
                    const int32_t c = A.col[e];
                    if (c >= lo && c < hi) kids_begin_[c + 1]++;
                }
        });
        std::partial_sum(kids_begin_.begin(), kids_begin_.end(), kids_begin_.begin());
        kids_.resize(kids_begin_[n]);
        parallel_rows(nw, n, [&](int64_t lo, int64_t hi) {
            std::vector<int64_t> pos(kids_begin_.begin() + lo, kids_begin_.begin() + hi);
            for (int64_t v = lo + 1; v < n; v++)
                for (int64_t e = A.row_ptr[v]; e < A.row_ptr[v + 1] - 1; e++) {
                    const int32_t c = A.col[e];
                    if (c >= lo && c < hi) kids_[pos[c - lo]++] = int32_t(v);
                }
        });
        work_.resize(size_t(nw));
        for (Worker &w : work_) w.tmp.assign(n, Tmp{0u, 0, 0});
        for (int64_t v = 0; v < n; v++)
            if (waiting_[v] == 0) free_.push_back(int32_t(v));
        for (size_t i = 1; i < work_.size(); i++) threads_.emplace_back([this, i] { serve(i); });
    }

    ~GrowLocalScheduler()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            quit_ = true;
        }
        cv_go_.notify_all();
        for (std::thread &t : threads_) t.join();
    }

    Schedule run()
    {
        Schedule out;
        out.core.assign(A_.n, -1);
        out.superstep.assign(A_.n, -1);
        int64_t done = 0;
        int32_t s = 0;
        const int width = int(work_.size());
        while (done < A_.n) {
            // grow alpha while the iterations stay worthy (Algorithm 3.1),
            // `width` iterations per round
            double alpha = p_.alpha0, best = 0.0;
            int it = 0;
            bool stop = false;
            while (!stop) {
                for (int i = 0; i < width; i++) {
                    work_[i].alpha = alpha;
                    alpha = p_.growth * alpha;
                }
                run_jobs(kTrial);
                int kept = -1;
                for (int i = 0; i < width; i++, it++) {
                    const Worker &w = work_[i];
                    const bool worthy = (it == 0) || (w.beta >= p_.accept * best);
                    if (!worthy) {
                        stop = true;
                        break;
                    }
                    kept = i;
                    if (it == 0 || w.beta > best) best = w.beta;
                    if (w.first_count < int64_t(std::floor(w.alpha))) {  // saturated
                        stop = true;
                        break;
                    }
                }
                if (kept >= 0) {
                    win_v_.swap(work_[kept].pv);
                    win_p_.swap(work_[kept].pp);
                }
            }
            for (size_t i = 0; i < win_v_.size(); i++) {
                out.core[win_v_[i]] = win_p_[i];
                out.superstep[win_v_[i]] = s;
            }
            out_ = &out;
            run_jobs(kCommit);
            merge_free(out);
            done += int64_t(win_v_.size());
            s++;
        }
        out.S = s;
        return out;
    }

private:
    struct Tmp {
        uint32_t epoch;
        int32_t wait, owner;  // unassigned parents left; core of the parents placed (-2: several)
    };
    struct Worker {
        std::vector<Tmp> tmp;         // trial fields valid where epoch matches
        uint32_t epoch = 0;
        std::vector<int32_t> excl;    // min-heap of vertices exclusive to the core
        std::vector<int32_t> pv, pp;  // picks (vertex, core) of its iteration
        std::vector<int32_t> fresh;   // children freed by its part of a commit
        double alpha = 0.0, beta = 0.0;
        int64_t first_count = 0;
    };
    enum Job { kTrial, kCommit };

    // One iteration from the barrier state with w.alpha.
    void trial(Worker &w)
    {
        if (++w.epoch == 0) {  // wrapped: forget every stale mark
            for (Tmp &m : w.tmp) m.epoch = 0;
            w.epoch = 1;
        }
        w.pv.clear();
        w.pp.clear();
        const int64_t limit = int64_t(std::floor(w.alpha));
        size_t next_free = 0;
        int64_t w_first = 0, total = 0, heaviest = 0, first_count = 0;
        for (int32_t core = 0; core < p_.k; core++) {
            w.excl.clear();
            int64_t count = 0, load = 0;
            while (core == 0 ? count < limit : load < w_first) {
                int32_t v;
                if (!w.excl.empty()) {
                    std::pop_heap(w.excl.begin(), w.excl.end(), std::greater<int32_t>());
                    v = w.excl.back();
                    w.excl.pop_back();
                } else if (next_free < free_.size()) {
                    v = free_[next_free++];
                } else {
                    break;
                }
                w.pv.push_back(v);
                w.pp.push_back(core);
                count++;
                load += weight_[v];
                for (int64_t e = kids_begin_[v]; e < kids_begin_[v + 1]; e++) {
                    const int32_t u = kids_[e];
                    Tmp &m = w.tmp[u];
                    if (m.epoch != w.epoch) {
                        m.epoch = w.epoch;
                        m.wait = waiting_[u];
                        m.owner = core;         // first parent placed in this superstep
                    } else if (m.owner != core) {
                        m.owner = -2;           // parents on two or more cores
                    }
                    if (--m.wait == 0 && m.owner == core) {
                        w.excl.push_back(u);
                        std::push_heap(w.excl.begin(), w.excl.end(), std::greater<int32_t>());
                    }
                }
            }
            if (core == 0) {
                w_first = load;
                first_count = count;
            }
            total += load;
            heaviest = std::max(heaviest, load);
            if (next_free >= free_.size()) break;  // nothing left for later cores
        }
        w.beta = double(total) / (double(heaviest) + p_.L);
        w.first_count = first_count;
    }

    // The committed superstep's vertices release their children; worker i
    // takes every nw-th slice of them and collects the children that became
    // free.
    void commit(size_t i)
    {
        const size_t nw = work_.size(), m = win_v_.size();
        std::vector<int32_t> &fresh = work_[i].fresh;
        fresh.clear();
        for (size_t q = i * m / nw; q < (i + 1) * m / nw; q++) {
            const int32_t v = win_v_[q];
            for (int64_t e = kids_begin_[v]; e < kids_begin_[v + 1]; e++) {
                const int32_t u = kids_[e];
                const int32_t left = nw > 1 ? __atomic_sub_fetch(&waiting_[u], 1, __ATOMIC_RELAXED) : --waiting_[u];
                if (left == 0 && out_->superstep[u] < 0) fresh.push_back(u);
            }
        }
    }

    void merge_free(const Schedule &out)
    {
        fresh_.clear();
        for (const Worker &w : work_) fresh_.insert(fresh_.end(), w.fresh.begin(), w.fresh.end());
        std::sort(fresh_.begin(), fresh_.end());
        merged_.clear();
        merged_.reserve(free_.size() + fresh_.size());
        auto keep = [&](int32_t v) { return out.superstep[v] < 0; };
        size_t a = 0, b = 0;
        while (a < free_.size() || b < fresh_.size()) {
            if (a < free_.size() && !keep(free_[a])) { a++; continue; }
            if (b == fresh_.size() || (a < free_.size() && free_[a] < fresh_[b])) merged_.push_back(free_[a++]);
            else merged_.push_back(fresh_[b++]);
        }
        free_.swap(merged_);
    }

    void do_job(size_t i)
    {
        if (job_ == kTrial) trial(work_[i]);
        else commit(i);
    }

    // Runs the job on every worker (worker 0 on the calling thread).
    void run_jobs(Job j)
    {
        if (threads_.empty()) {
            job_ = j;
            do_job(0);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            job_ = j;
            pending_ = int(threads_.size());
            gen_++;
        }
        cv_go_.notify_all();
        do_job(0);
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.wait(lk, [&] { return pending_ == 0; });
    }

    void serve(size_t i)
    {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_go_.wait(lk, [&] { return quit_ || gen_ != seen; });
                if (quit_) return;
                seen = gen_;
            }
            do_job(i);
            std::lock_guard<std::mutex> g(mu_);
            if (--pending_ == 0) cv_done_.notify_one();
        }
    }

    const CsrView &A_;
    SchedParams p_;
    std::vector<int64_t> weight_;
    std::vector<int32_t> waiting_;     // unassigned parents at the barrier
    std::vector<int64_t> kids_begin_;
    std::vector<int32_t> kids_;
    std::vector<int32_t> free_;        // free at the barrier, rising IDs
    std::vector<int32_t> fresh_, merged_;
    std::vector<int32_t> win_v_, win_p_;  // picks of the kept iteration
    std::vector<Worker> work_;
    const Schedule *out_ = nullptr;
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable cv_go_, cv_done_;
    Job job_ = kTrial;
    uint64_t gen_ = 0;
    int pending_ = 0;
    bool quit_ = false;
};

}  // namespace

int growlocal_workers(int64_t n, int32_t requested)
{
    if (requested > 0) return requested;
    if (n < 200000) return 1;
    const int hw = int(std::max(1u, std::thread::hardware_concurrency()));
    const int64_t by_mem = std::max<int64_t>(1, (int64_t(4) << 30) / (16 * n));  // trial state <= 4 GiB
    return int(std::min<int64_t>({8, hw, by_mem}));
}

std::vector<int64_t> block_bounds(int64_t n, int32_t nblocks)
{
    std::vector<int64_t> b(size_t(nblocks) + 1);
    for (int32_t i = 0; i <= nblocks; i++) b[size_t(i)] = (int64_t(i) * n) / nblocks;
    return b;
}

namespace {

// Block-parallel GrowLocal (Sec. 3.1): every diagonal block is its own DAG
// (edges from earlier blocks dropped; those parents finish in earlier
// supersteps) scheduled with the weights of the full rows, the blocks on
// separate threads; superstep numbers are then offset block after block.
Schedule schedule_growlocal_blocks(const CsrView &A, const SchedParams &p)
{
    const int64_t n = A.n;
    const int32_t nb = p.blocks;
    const std::vector<int64_t> bounds = block_bounds(n, nb);
    std::vector<Schedule> part(static_cast<size_t>(nb));
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        for (int32_t b; (b = next.fetch_add(1)) < nb;) {
            const int64_t lo = bounds[size_t(b)], hi = bounds[size_t(b) + 1];
            if (hi == lo) continue;
            std::vector<int64_t> rp(size_t(hi - lo) + 1, 0), w(size_t(hi - lo));
            std::vector<int32_t> col;
            col.reserve(size_t(A.row_ptr[hi] - A.row_ptr[lo]));
            for (int64_t i = lo; i < hi; i++) {
                for (int64_t e = A.row_ptr[i]; e < A.row_ptr[i + 1]; e++)
                    if (A.col[e] >= lo) col.push_back(int32_t(A.col[e] - lo));
                rp[size_t(i - lo) + 1] = int64_t(col.size());
                w[size_t(i - lo)] = A.row_ptr[i + 1] - A.row_ptr[i];
            }
            CsrView sub;
            sub.n = hi - lo;
            sub.nnz = int64_t(col.size());
            sub.row_ptr = rp.data();
            sub.col = col.data();
            GrowLocalScheduler g(sub, p, 1, w.data());
            part[size_t(b)] = g.run();
        }
    };
    const int threads = std::max(1, std::min<int>(nb, growlocal_workers(n, p.threads)));
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; t++) pool.emplace_back(worker);
    worker();
    for (std::thread &t : pool) t.join();
    Schedule out;
    out.core.resize(size_t(n));
    out.superstep.resize(size_t(n));
    int32_t offset = 0;
    for (int32_t b = 0; b < nb; b++) {
        const int64_t lo = bounds[size_t(b)], hi = bounds[size_t(b) + 1];
        for (int64_t i = lo; i < hi; i++) {
            out.core[size_t(i)] = part[size_t(b)].core[size_t(i - lo)];
            out.superstep[size_t(i)] = part[size_t(b)].superstep[size_t(i - lo)] + offset;
        }
        offset += part[size_t(b)].S;
    }
    out.S = offset;
    return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Funnel coarsening (Sec. 4)
// ---------------------------------------------------------------------------

ReducedDag transitive_reduction(const CsrView &A)
{
    const int64_t n = A.n;
    // children lists, rising
    std::vector<int64_t> cb(size_t(n) + 1, 0);
    for (int64_t w = 0; w < n; w++)
        for (int64_t e = A.row_ptr[w]; e < A.row_ptr[w + 1] - 1; e++) cb[size_t(A.col[e]) + 1]++;
    std::partial_sum(cb.begin(), cb.end(), cb.begin());
    std::vector<int32_t> ch(size_t(cb[size_t(n)]));
    {
        std::vector<int64_t> pos(cb.begin(), cb.end() - 1);
        for (int64_t w = 0; w < n; w++)
            for (int64_t e = A.row_ptr[w]; e < A.row_ptr[w + 1] - 1; e++) ch[size_t(pos[size_t(A.col[e])]++)] = int32_t(w);
    }
    ReducedDag r;
    r.beg.assign(size_t(n) + 1, 0);
    r.par.reserve(size_t(A.nnz - n));
    std::vector<int32_t> mark(size_t(n), -1);   // mark[u] == w: u is a parent of w
    for (int64_t w = 0; w < n; w++) {
        const int64_t lo = A.row_ptr[w], hi = A.row_ptr[w + 1] - 1;
        for (int64_t e = lo; e < hi; e++) mark[size_t(A.col[e])] = int32_t(w);
        for (int64_t e = lo; e < hi; e++) {
            const int32_t u = A.col[e];
            bool is_long = false;   // u -> v -> w for some parent v of w
            for (int64_t q = cb[size_t(u)]; q < cb[size_t(u) + 1]; q++) {
                const int32_t v = ch[size_t(q)];
                if (v >= w) break;
                if (mark[size_t(v)] == int32_t(w)) {
                    is_long = true;
                    break;
                }
            }
            if (!is_long) r.par.push_back(u);
        }
        r.beg[size_t(w) + 1] = int64_t(r.par.size());
    }
    return r;
}

std::vector<int32_t> funnel_partition(const CsrView &A, const ReducedDag &r, int64_t max_weight, int32_t *nparts)
{
    const int64_t n = A.n;
    std::vector<int32_t> outdeg(size_t(n), 0);
    for (int32_t u : r.par) outdeg[size_t(u)]++;
    std::vector<char> visited(size_t(n), 0);
    std::vector<int32_t> count(size_t(n), 0), touched, members, root_of(size_t(n), -1);
    std::priority_queue<int32_t> heap;   // largest vertex first
    int32_t parts = 0;
    for (int64_t v = n - 1; v >= 0; v--) {
        if (visited[size_t(v)]) continue;
        members.clear();
        int64_t weight = 0;
        heap.push(int32_t(v));
        while (!heap.empty()) {
            const int32_t x = heap.top();
            heap.pop();
            const int64_t wx = A.row_ptr[x + 1] - A.row_ptr[x];
            if (weight + wx > max_weight && !members.empty()) continue;   // over the cap
            members.push_back(x);
            weight += wx;
            for (int64_t e = r.beg[size_t(x)]; e < r.beg[size_t(x) + 1]; e++) {
                const int32_t u = r.par[size_t(e)];
                if (count[size_t(u)]++ == 0) touched.push_back(u);
                if (count[size_t(u)] == outdeg[size_t(u)]) heap.push(u);
            }
        }
        for (int32_t u : touched) count[size_t(u)] = 0;
        touched.clear();
        for (int32_t x : members) {
            visited[size_t(x)] = 1;
            root_of[size_t(x)] = parts;   // discovery index; roots fall, so parts renumber below
        }
        parts++;
    }
    // parts numbered by root in rising order (a topological order of the coarsened DAG)
    for (int32_t &q : root_of) q = parts - 1 - q;
    *nparts = parts;
    return root_of;
}

namespace {

Schedule schedule_funnel_growlocal(const CsrView &A, const SchedParams &p)
{
    const int64_t n = A.n;
    const ReducedDag r = transitive_reduction(A);
    int32_t P = 0;
    const std::vector<int32_t> part = funnel_partition(A, r, p.funnel_max_weight, &P);
    // coarsened DAG (Definition 4.1) of the reduced DAG, as a lower pattern
    std::vector<std::pair<int32_t, int32_t>> edges;   // (part of child, part of parent)
    std::vector<int64_t> weight(size_t(P), 0);
    for (int64_t w = 0; w < n; w++) {
        weight[size_t(part[size_t(w)])] += A.row_ptr[w + 1] - A.row_ptr[w];
        for (int64_t e = r.beg[size_t(w)]; e < r.beg[size_t(w) + 1]; e++) {
            const int32_t u = r.par[size_t(e)];
            if (part[size_t(u)] != part[size_t(w)]) edges.emplace_back(part[size_t(w)], part[size_t(u)]);
        }
    }
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    std::vector<int64_t> crp(size_t(P) + 1, 0);
    std::vector<int32_t> ccol;
    ccol.reserve(edges.size() + size_t(P));
    size_t q = 0;
    for (int32_t c = 0; c < P; c++) {
        while (q < edges.size() && edges[q].first == c) ccol.push_back(edges[q++].second);
        ccol.push_back(c);
        crp[size_t(c) + 1] = int64_t(ccol.size());
    }
    CsrView cv;
    cv.n = P;
    cv.nnz = int64_t(ccol.size());
    cv.row_ptr = crp.data();
    cv.col = ccol.data();
    GrowLocalScheduler g(cv, p, growlocal_workers(P, p.threads), weight.data());
    const Schedule cs = g.run();
    Schedule out;
    out.core.resize(size_t(n));
    out.superstep.resize(size_t(n));
    for (int64_t v = 0; v < n; v++) {
        out.core[size_t(v)] = cs.core[size_t(part[size_t(v)])];
        out.superstep[size_t(v)] = cs.superstep[size_t(part[size_t(v)])];
    }
    out.S = cs.S;
    return out;
}

}  // namespace

Schedule schedule_growlocal(const CsrView &A, const SchedParams &p)
{
    if (A.n == 0) return Schedule{};
    if (p.funnel_max_weight > 0) return schedule_funnel_growlocal(A, p);
    if (p.blocks > 1) return schedule_growlocal_blocks(A, p);
    GrowLocalScheduler g(A, p, growlocal_workers(A.n, p.threads));
    return g.run();
}

std::vector<int32_t> schedule_order(int64_t n, const int32_t *core, const int32_t *superstep, int32_t S)
{
    // two stable counting passes: by core, then by superstep
    int32_t kmax = 0;
    for (int64_t i = 0; i < n; i++) kmax = std::max(kmax, core[i]);
    std::vector<int64_t> cnt(std::max<int64_t>(kmax + 1, S) + 1, 0);
    std::vector<int32_t> by_core(n), out(n);
    for (int64_t i = 0; i < n; i++) cnt[core[i] + 1]++;
    for (size_t c = 1; c < cnt.size(); c++) cnt[c] += cnt[c - 1];
    for (int64_t i = 0; i < n; i++) by_core[cnt[core[i]]++] = int32_t(i);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t i = 0; i < n; i++) cnt[superstep[i] + 1]++;
    for (size_t c = 1; c < cnt.size(); c++) cnt[c] += cnt[c - 1];
    for (int64_t t = 0; t < n; t++) {
        const int32_t v = by_core[t];
        out[cnt[superstep[v]]++] = v;
    }
    return out;
}

PackLayout pack_layout(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm)
{
    PackLayout lay;
    Packed &pk = lay.pk;
    pk.S = sch.S;
    const int64_t n = A.n;
    // tasks = maximal runs of equal (superstep, core) in the order
    std::vector<int64_t> task_begin;
    for (int64_t t = 0; t < n; t++) {
        const int32_t v = perm[t];
        if (t == 0 || sch.superstep[v] != sch.superstep[perm[t - 1]] || sch.core[v] != sch.core[perm[t - 1]])
            task_begin.push_back(t);
    }
    const int64_t T = int64_t(task_begin.size());
    task_begin.push_back(n);
    pk.tasks = T;
    std::vector<int64_t> task_len(T);  // stream entries = stored entries of its rows
    for (int64_t j = 0; j < T; j++) {
        int64_t e = 0;
        for (int64_t t = task_begin[j]; t < task_begin[j + 1]; t++) e += A.row_ptr[perm[t] + 1] - A.row_ptr[perm[t]];
        task_len[j] = e;
        pk.max_task_rows = std::max(pk.max_task_rows, task_begin[j + 1] - task_begin[j]);
    }
    // per superstep: tasks longest first, 64 per chunk
    pk.super_chunk.assign(sch.S + 1, 0);
    std::vector<int64_t> order;
    std::vector<int64_t> lane_task;  // task of each (chunk, lane), -1 for none
    int64_t j0 = 0;
    for (int32_t s = 0; s < sch.S; s++) {
        int64_t j1 = j0;
        while (j1 < T && sch.superstep[perm[task_begin[j1]]] == s) j1++;
        order.resize(j1 - j0);
        std::iota(order.begin(), order.end(), j0);
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return task_len[a] > task_len[b]; });
        for (size_t q = 0; q < order.size(); q += kLanes) {
            int64_t len = 0;
            for (size_t l = 0; l < size_t(kLanes); l++) {
                const int64_t task = (q + l < order.size()) ? order[q + l] : -1;
                lane_task.push_back(task);
                if (task >= 0) len = std::max(len, task_len[task]);
            }
            pk.chunk_len.push_back(int32_t(len));
        }
        pk.super_chunk[s + 1] = int32_t(pk.chunk_len.size());
        j0 = j1;
    }
    const int64_t C = int64_t(pk.chunk_len.size());
    pk.chunk_base.resize(C);
    int64_t slots = 0;
    for (int64_t c = 0; c < C; c++) {
        pk.chunk_base[c] = slots;
        slots += int64_t(kLanes) * pk.chunk_len[c];
    }
    pk.slots = slots;
    lay.pos_slot.assign(n, 0);
    lay.pos_task0.assign(n, 0);
    lay.lane_first.assign(size_t(C) * kLanes, 0);
    lay.lane_rows.assign(size_t(C) * kLanes, 0);
    for (int64_t c = 0; c < C; c++) {
        for (int l = 0; l < kLanes; l++) {
            const int64_t task = lane_task[c * kLanes + l];
            if (task < 0) continue;
            lay.lane_first[size_t(c * kLanes + l)] = int32_t(task_begin[task]);
            lay.lane_rows[size_t(c * kLanes + l)] = int32_t(task_begin[task + 1] - task_begin[task]);
            for (int64_t t = task_begin[task]; t < task_begin[task + 1]; t++) {
                lay.pos_slot[t] = pk.chunk_base[c] + l;
                lay.pos_task0[t] = int32_t(task_begin[task]);
            }
        }
    }
    return lay;
}

void pack_fill(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm, PackLayout &lay)
{
    Packed &pk = lay.pk;
    const int64_t n = A.n;
    pk.word.assign(pk.slots, kPadWord);
    pk.value.assign(pk.slots, 0.0);
    std::vector<int32_t> inv(n);
    for (int64_t t = 0; t < n; t++) inv[perm[t]] = int32_t(t);
    int64_t off = 0;   // entries of the current task before position t
    for (int64_t t = 0; t < n; t++) {
        if (t == lay.pos_task0[t]) off = 0;
        const int32_t row = perm[t];
        const int64_t lo = A.row_ptr[row], hi = A.row_ptr[row + 1] - 1;
        const int64_t base = lay.pos_slot[t];
        pk.word[base + int64_t(kLanes) * off] = kHdrBit | uint32_t(row);
        pk.value[base + int64_t(kLanes) * off] = A.val ? A.val[hi] : 1.0;
        for (int64_t e = lo; e < hi; e++) {
            const int32_t col = A.col[e];
            uint32_t w = uint32_t(col);
            if (sch.superstep[col] == sch.superstep[row] && sch.core[col] == sch.core[row]) {
                const int64_t back = t - inv[col];   // rows back inside the task
                if (back < kRing) w = kIntBit | uint32_t(back);
            }
            const int64_t at = base + int64_t(kLanes) * (off + 1 + (e - lo));
            pk.word[at] = w;
            pk.value[at] = A.val ? A.val[e] : 0.0;
        }
        off += hi - lo + 1;
    }
}

void pack_fill_upper(const CsrView &U, const std::vector<int32_t> &perm, PackLayout &lay)
{
    Packed &pk = lay.pk;
    const int64_t n = U.n;
    pk.word.assign(pk.slots, kPadWord);
    pk.value.assign(pk.slots, 0.0);
    std::vector<int32_t> inv(n);
    for (int64_t t = 0; t < n; t++) inv[perm[t]] = int32_t(t);
    int64_t off = 0;
    for (int64_t t = 0; t < n; t++) {
        if (t == lay.pos_task0[t]) off = 0;
        const int64_t i = n - 1 - perm[t];
        const int64_t lo = U.row_ptr[i], hi = U.row_ptr[i + 1];   // diagonal at lo
        const int64_t base = lay.pos_slot[t];
        pk.word[base + int64_t(kLanes) * off] = kHdrBit | uint32_t(i);
        pk.value[base + int64_t(kLanes) * off] = U.val[lo];
        for (int64_t e = lo + 1; e < hi; e++) {
            const int32_t col = U.col[e];
            uint32_t w = uint32_t(col);
            const int64_t ic = inv[n - 1 - col];
            // a parent at or after the task's first position is in this task
            if (ic >= lay.pos_task0[t] && t - ic < kRing) w = kIntBit | uint32_t(t - ic);
            const int64_t at = base + int64_t(kLanes) * (off + (e - lo));
            pk.word[at] = w;
            pk.value[at] = U.val[e];
        }
        off += hi - lo;
    }
}

Packed pack_stream(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm)
{
    PackLayout lay = pack_layout(A, sch, perm);
    pack_fill(A, sch, perm, lay);
    return std::move(lay.pk);
}

double predict_cost_us(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm, const CostModel &cm)
{
    double total = 0.0;
    int64_t t = 0;
    const int64_t n = A.n;
    while (t < n) {
        const int32_t s = sch.superstep[perm[t]];
        int64_t longest = 0, entries = 0;
        while (t < n && sch.superstep[perm[t]] == s) {
            const int32_t p = sch.core[perm[t]];
            int64_t task = 0;
            while (t < n && sch.superstep[perm[t]] == s && sch.core[perm[t]] == p) {
                task += A.row_ptr[perm[t] + 1] - A.row_ptr[perm[t]];
                t++;
            }
            longest = std::max(longest, task);
            entries += task;
        }
        total += cm.superstep_us + std::max(cm.entry_us * double(longest), double(entries) / cm.entries_per_us);
    }
    return total;
}

double predict_async_us(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm, const CostModel &cm)
{
    const int64_t n = A.n;
    std::vector<double> finish(size_t(n), 0.0);
    double path = 0.0;
    for (int64_t t = 0; t < n; t++) {
        const int32_t i = perm[size_t(t)];
        const bool same = t > 0 && sch.superstep[size_t(perm[size_t(t - 1)])] == sch.superstep[size_t(i)] &&
                          sch.core[size_t(perm[size_t(t - 1)])] == sch.core[size_t(i)];
        double start = same ? finish[size_t(perm[size_t(t - 1)])] : 0.0;
        for (int64_t e = A.row_ptr[i]; e < A.row_ptr[i + 1] - 1; e++) {
            const int32_t j = A.col[e];
            if (sch.superstep[size_t(j)] != sch.superstep[size_t(i)] || sch.core[size_t(j)] != sch.core[size_t(i)])
                start = std::max(start, finish[size_t(j)] + cm.hop_us);
        }
        finish[size_t(i)] = start + cm.entry_us * double(A.row_ptr[i + 1] - A.row_ptr[i]);
        path = std::max(path, finish[size_t(i)]);
    }
    return cm.launch_us + std::max(path, double(A.nnz) / cm.entries_per_us);
}

uint64_t pattern_key(const CsrView &A)
{
    // 64-bit multiply-xorshift mix over n, row pointers and columns
    uint64_t h = 0x9E3779B97F4A7C15ull ^ uint64_t(A.n);
    auto mix = [&](uint64_t x) {
        h ^= x + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 31;
    };
    for (int64_t i = 0; i <= A.n; i++) mix(uint64_t(A.row_ptr[i]));
    for (int64_t e = 0; e + 1 < A.nnz; e += 2) mix(uint64_t(uint32_t(A.col[e])) | (uint64_t(uint32_t(A.col[e + 1])) << 32));
    if (A.nnz & 1) mix(uint64_t(uint32_t(A.col[A.nnz - 1])));
    return h;
}

}  // namespace gltrsv
