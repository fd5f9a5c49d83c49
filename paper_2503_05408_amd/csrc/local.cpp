// Host side of single-workgroup execution: the groups, records and FIFO
// placement described in local.h.
#include "local.h"

#include <algorithm>
#include <cstring>

#include "../../include/gltrsv.h"

namespace gltrsv {

namespace {

inline uint64_t align16(uint64_t b) { return (b + 15) & ~uint64_t(15); }
inline uint64_t align_block(uint64_t b) { return (b + kLocalAlign - 1) & ~uint64_t(kLocalAlign - 1); }

// FIFO bytes of a record: the copied part, then its staging slots in whole
// blocks of 64 from the next block boundary.
inline uint64_t copied_bytes(int64_t groups, int64_t fills, int64_t drains)
{
    return align16(uint64_t(kLocalHdrBytes) + uint64_t(kLocalGroupBytes) * uint64_t(groups) + 8 * uint64_t(fills) +
                   8 * uint64_t(drains));
}
inline uint64_t footprint(int64_t groups, int64_t fills, int64_t drains)
{
    return align_block(copied_bytes(groups, fills, drains)) + align_block(8 * uint64_t(fills));
}

struct Fill {
    int64_t entry;     // (group * 64 + lane) * 4 + slot of the entry that reads it
    int32_t row;       // b[row] or x[row]
    int64_t source;    // for x: the group where row's value was computed; -1 for b
};

}  // namespace

int64_t local_group_count(const CsrView &D, const Schedule &sch, const std::vector<int32_t> &perm)
{
    const int64_t n = D.n;
    int64_t total = 0, lane_groups[64];
    for (int64_t p = 0; p < n;) {
        const int32_t s = sch.superstep[size_t(perm[size_t(p)])];
        std::fill(lane_groups, lane_groups + 64, int64_t(0));
        for (; p < n && sch.superstep[size_t(perm[size_t(p)])] == s; p++) {
            const int32_t v = perm[size_t(p)];
            lane_groups[sch.core[size_t(v)] & 63] += (D.row_ptr[v + 1] - D.row_ptr[v] + 3) / 4;
        }
        total += *std::max_element(lane_groups, lane_groups + 64);
    }
    return total;
}

void fold_cores(Schedule &sch, int32_t cores)
{
    for (int32_t &c : sch.core) c %= cores;
}

int build_local_layout(const CsrView &A, bool upper, const Schedule &sch, const std::vector<int32_t> &perm,
                       LocalLayout *out, std::string *msg)
{
    const int64_t n = A.n;
    auto row_of = [&](int64_t v) { return upper ? n - 1 - v : v; };
    auto len_of = [&](int64_t v) {
        const int64_t r = row_of(v);
        return A.row_ptr[r + 1] - A.row_ptr[r];
    };

    // 1. groups: lane c walks its rows of superstep s in the order of Sec. 5,
    // ceil(entries / 4) groups per row; superstep s takes as many groups as
    // its busiest lane
    std::vector<int64_t> gfirst(static_cast<size_t>(n)), glast(static_cast<size_t>(n));
    int64_t gbase = 0;
    int64_t lane_groups[64];
    for (int64_t p = 0; p < n;) {
        const int32_t s = sch.superstep[size_t(perm[size_t(p)])];
        std::fill(lane_groups, lane_groups + 64, int64_t(0));
        for (; p < n && sch.superstep[size_t(perm[size_t(p)])] == s; p++) {
            const int32_t v = perm[size_t(p)];
            const int32_t c = sch.core[size_t(v)];
            if (c < 0 || c >= 64) {
                *msg = "single-workgroup execution needs cores 0..63 (k <= 64); core " + std::to_string(c);
                return GLTRSV_EINVAL;
            }
            const int64_t ng = (len_of(v) + 3) / 4;
            gfirst[size_t(v)] = gbase + lane_groups[c];
            lane_groups[c] += ng;
            glast[size_t(v)] = gfirst[size_t(v)] + ng - 1;
        }
        gbase += *std::max_element(lane_groups, lane_groups + 64);
    }
    const int64_t G = gbase;

    // 2. entries: operand slot (u16) and value per (group, lane, entry);
    // padding reads the zero slot with value 0 (acc - 0 * 0 = acc, bit for bit)
    std::vector<uint16_t> opa(size_t(G) * 256, uint16_t(kLocalZeroSlot));
    std::vector<double> val(size_t(G) * 256, 0.0);
    std::vector<Fill> fills;
    fills.reserve(size_t(n) + size_t(n) / 4);
    std::vector<std::pair<int64_t, int32_t>> drains;   // (group * 64 + lane, row)
    drains.reserve(size_t(n));
    int64_t far = 0;
    for (int64_t v = 0; v < n; v++) {
        const int64_t lane = sch.core[size_t(v)];
        const int64_t row = row_of(v);
        const int64_t beg = A.row_ptr[row], end = A.row_ptr[row + 1];
        const int64_t dpos = upper ? beg : end - 1;
        // header: diagonal, b[row] staged
        const int64_t e0 = (gfirst[size_t(v)] * 64 + lane) * 4;
        val[size_t(e0)] = A.val[dpos];
        fills.push_back(Fill{e0, int32_t(row), -1});
        // off-diagonals in stored order
        int64_t j = 1;
        for (int64_t k = upper ? beg + 1 : beg; k < (upper ? end : end - 1); k++, j++) {
            const int64_t g = gfirst[size_t(v)] + j / 4;
            const int64_t e = (g * 64 + lane) * 4 + j % 4;
            const int64_t u = upper ? n - 1 - A.col[k] : A.col[k];
            const int64_t gp = glast[size_t(u)];
            val[size_t(e)] = A.val[k];
            if (g - gp < kLocalRingGroups) {
                opa[size_t(e)] = uint16_t((gp % kLocalRingGroups) * 64 + sch.core[size_t(u)]);
            } else {
                fills.push_back(Fill{e, int32_t(row_of(u)), gp});
                far++;
            }
        }
        const int64_t el = glast[size_t(v)] * 64 + lane;
        opa[size_t(el * 4 + 1)] |= uint16_t(kLocalEndBit);
        drains.emplace_back(el, int32_t(row));
    }
    std::stable_sort(fills.begin(), fills.end(), [](const Fill &a, const Fill &b) { return a.entry < b.entry; });
    std::sort(drains.begin(), drains.end());

    // 3. records: consecutive groups while the FIFO footprint stays within
    // kLocalRecMax
    std::vector<int64_t> gfill(size_t(G) + 1, 0), gdrain(size_t(G) + 1, 0);
    for (const Fill &f : fills) gfill[size_t(f.entry / 256) + 1]++;
    for (const auto &d : drains) gdrain[size_t(d.first / 64) + 1]++;
    for (int64_t g = 0; g < G; g++) {
        gfill[size_t(g) + 1] += gfill[size_t(g)];
        gdrain[size_t(g) + 1] += gdrain[size_t(g)];
    }
    std::vector<int64_t> rfirst;   // first group of each record
    for (int64_t g = 0; g < G;) {
        rfirst.push_back(g);
        int64_t h = g + 1;
        while (h < G && h - g < kLocalRingGroups / 2 &&
               footprint(h + 1 - g, gfill[size_t(h) + 1] - gfill[size_t(g)], gdrain[size_t(h) + 1] - gdrain[size_t(g)]) <=
                   uint64_t(kLocalRecMax))
            h++;
        g = h;
    }
    const int64_t R = int64_t(rfirst.size());
    rfirst.push_back(G);
    std::vector<int32_t> rec_of(static_cast<size_t>(G));
    for (int64_t r = 0; r < R; r++)
        for (int64_t g = rfirst[size_t(r)]; g < rfirst[size_t(r) + 1]; g++) rec_of[size_t(g)] = int32_t(r);

    // 4. FIFO placement: one record after another, back to 0 when the next
    // does not fit; a record waits until every earlier record whose bytes it
    // reuses is computed
    std::vector<uint32_t> foff(static_cast<size_t>(R)), fsize(static_cast<size_t>(R)), cbytes(static_cast<size_t>(R));
    out->info.assign(size_t(R), LocalRec{});
    uint64_t at = 0;
    for (int64_t r = 0; r < R; r++) {
        const int64_t g0 = rfirst[size_t(r)], g1 = rfirst[size_t(r) + 1];
        const int64_t nf = gfill[size_t(g1)] - gfill[size_t(g0)], nd = gdrain[size_t(g1)] - gdrain[size_t(g0)];
        const uint64_t fp = footprint(g1 - g0, nf, nd);
        if (at + fp > uint64_t(kLocalFifoBytes)) at = 0;
        foff[size_t(r)] = uint32_t(at);
        fsize[size_t(r)] = uint32_t(fp);
        cbytes[size_t(r)] = uint32_t(copied_bytes(g1 - g0, nf, nd));
        at += fp;
        uint32_t wait = 0;
        for (int64_t q = r - 1; q >= 0; q--) {
            if (foff[size_t(q)] < foff[size_t(r)] + fsize[size_t(r)] && foff[size_t(r)] < foff[size_t(q)] + fsize[size_t(q)]) {
                wait = uint32_t(q + 1);
                break;
            }
            if (r - q > 2 * (kLocalFifoBytes / (kLocalHdrBytes + kLocalGroupBytes)) + 2) break;
        }
        LocalRec &info = out->info[size_t(r)];
        info.bytes = cbytes[size_t(r)];
        info.fifo_off = foff[size_t(r)];
        info.wait = wait;
        info.unused = 0;
    }

    // 5. fill slots, far dependencies, records
    uint64_t total = 0;
    for (int64_t r = 0; r < R; r++) total += cbytes[size_t(r)];
    out->rec.assign(total, 0);
    uint64_t w = 0;
    for (int64_t r = 0; r < R; r++) {
        const int64_t g0 = rfirst[size_t(r)], g1 = rfirst[size_t(r) + 1];
        const int64_t f0 = gfill[size_t(g0)], f1 = gfill[size_t(g1)];
        const int64_t d0 = gdrain[size_t(g0)], d1 = gdrain[size_t(g1)];
        const uint32_t slot0 = uint32_t(kLocalFifoSlot0) + uint32_t((foff[size_t(r)] + align_block(cbytes[size_t(r)])) / 8);
        uint32_t need_far = 0;
        for (int64_t i = f0; i < f1; i++) {
            const Fill &f = fills[size_t(i)];
            const uint32_t slot = slot0 + uint32_t(i - f0);
            const bool hdr = f.source < 0;
            // a header takes the start bit; an operand keeps the end bit of entry 1
            opa[size_t(f.entry)] = uint16_t(slot | (hdr ? kLocalStartBit : (opa[size_t(f.entry)] & kLocalEndBit)));
            if (!hdr) need_far = std::max(need_far, uint32_t(rec_of[size_t(f.source)] + 1));
        }
        // the ring slots written here last held the rows of group g - kLocalRingGroups
        const int64_t old = g1 - 1 - kLocalRingGroups;
        LocalHdr h{};
        h.ngroups = uint32_t(g1 - g0);
        h.nfill = uint32_t(f1 - f0);
        h.ndrain = uint32_t(d1 - d0);
        h.need_drain = old >= 0 ? uint32_t(rec_of[size_t(old)] + 1) : 0u;
        h.next_off = r + 1 < R ? foff[size_t(r) + 1] : 0u;
        h.need_far = need_far;
        uint8_t *o = out->rec.data() + w;
        std::memcpy(o, &h, sizeof(h));
        uint8_t *gp = o + kLocalHdrBytes;
        for (int64_t g = g0; g < g1; g++, gp += kLocalGroupBytes) {
            double *vv = reinterpret_cast<double *>(gp);
            uint16_t *oo = reinterpret_cast<uint16_t *>(gp + 2048);
            for (int l = 0; l < 64; l++) {
                const size_t e = size_t((g * 64 + l) * 4);
                vv[l * 2 + 0] = val[e + 0];
                vv[l * 2 + 1] = val[e + 1];
                vv[128 + l * 2 + 0] = val[e + 2];
                vv[128 + l * 2 + 1] = val[e + 3];
                for (int j = 0; j < 4; j++) oo[l * 4 + j] = opa[e + size_t(j)];
            }
        }
        uint32_t *fl = reinterpret_cast<uint32_t *>(gp);
        for (int64_t i = f0; i < f1; i++) {
            const Fill &f = fills[size_t(i)];
            fl[2 * (i - f0)] = (slot0 + uint32_t(i - f0)) | (f.source >= 0 ? kLocalFillX : 0u);
            fl[2 * (i - f0) + 1] = uint32_t(f.row);
        }
        uint32_t *dl = fl + 2 * (f1 - f0);
        for (int64_t i = d0; i < d1; i++) {
            const int64_t gl = drains[size_t(i)].first;
            dl[2 * (i - d0)] = uint32_t(((gl / 64) % kLocalRingGroups) * 64 + gl % 64);
            dl[2 * (i - d0) + 1] = uint32_t(drains[size_t(i)].second);
        }
        w += cbytes[size_t(r)];
    }
    out->groups = G;
    out->far = far;
    out->entries = G * 256;
    return 0;
}

}  // namespace gltrsv
