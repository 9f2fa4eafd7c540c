// Grouping of a column-sliced operator's segments into staged units for the
// LDS product kernel.  Host code only (no HIP): included by the C-ABI source
// and compiled on its own by a host test.
//
// A unit is a run of consecutive segments of one slice (consecutive rows)
// whose nonzeros read at most `cap` distinct source rows of the block X.  The
// kernel copies those rows into LDS once and streams the unit's records
// against the copy, so a source row read by several rows of the unit leaves L2
// once instead of once per nonzero.
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <vector>

namespace sfk {

struct UnitPlan {
  std::vector<int32_t> unit;    // 4 per unit: first segment, end segment, first staged row, staged rows
  std::vector<int32_t> stage;   // cap per unit: source row (block row of X) of each staged row,
                                // -1 past the unit's rows (unit u's list starts at u * cap)
  std::vector<int32_t> split;   // (ng + 1) per unit: segment range of each lane group
  std::vector<int32_t> group;   // 4 per unit and lane group: first segment, end segment,
                                // first record, end record (all 0 for an empty range)
  std::vector<int32_t> upart;   // NS * (nbw + 1): unit range of each workgroup of a slice
  std::vector<int32_t> off;     // byte offset of every record inside its unit's staged block
  std::vector<int32_t> endslot; // per record: partial slot of its segment if it is the
                                // segment's last record, else -1
  int64_t nonzeros = 0;         // records that are not padding
  int64_t staged = 0;           // staged rows over all units
  int max_records = 0;          // records of the largest unit
};

// Index q in [lo, hi] whose boundary pos(q) is nearest to target (pos is
// non-decreasing), the first such q on a tie.
template <class Pos>
inline int nearest_boundary(int lo, int hi, int64_t target, Pos pos) {
  int a = lo, b = hi;
  while (a < b) {               // first q with pos(q) >= target
    const int mid = (a + b) >> 1;
    if (pos(mid) < target) a = mid + 1; else b = mid;
  }
  if (a > lo && target - pos(a - 1) <= pos(a) - target) --a;
  return a;
}

// seg[4 q .. 4 q + 3] = (row, first record, end record, slot) of segment q,
// stored slice-major: slice s holds segments sbeg[s] .. sbeg[s + 1] - 1 in row
// order, and the records of consecutive segments are contiguous.  off[e] is the
// byte offset of record e's source row (source row * rowbytes), or padoff for
// a padding record.  In the plan, a record's offset is its source row's slot
// in the unit's staged block times rowbytes; padding and records outside every
// segment point at byte cap * rowbytes, a row of zeros after the block.  The
// last record of a segment carries the segment's partial slot (endslot).
// A unit holds at most nzcap records (padding included).
// ng lane groups share a unit (contiguous segment ranges, balanced by records);
// nbw workgroups share a slice (contiguous unit ranges, balanced by records +
// stage_weight * staged rows).
// Returns false (P cleared) when a segment reads more than cap distinct rows
// or holds more than nzcap records, or an offset is not a source row.
inline bool plan_units(int NS, const int32_t *sbeg, const int32_t *seg, const int32_t *off,
                       int64_t nrec, int cols, int rowbytes, int32_t padoff, int cap, int nzcap,
                       int ng, int nbw, int stage_weight, UnitPlan &P) {
  P = UnitPlan();
  const int32_t zero_row = cap * rowbytes;
  P.off.assign((size_t)nrec, zero_row);
  P.endslot.assign((size_t)nrec, -1);
  std::vector<int32_t> stamp(cols, -1), slot(cols, 0), seen(cols, -1);
  std::vector<int64_t> weight;  // per unit, for the workgroup split
  auto fail = [&P]() { P = UnitPlan(); return false; };
  auto rec_begin = [&](int q) { return (int64_t)seg[4 * (size_t)q + 1]; };

  int open = -1, first = 0, count = 0;
  auto close_unit = [&](int end) {
    if (open < 0) return;
    const int stage0 = (int)(P.stage.size() - count);
    P.stage.resize((size_t)stage0 + cap, -1);
    P.unit.insert(P.unit.end(), {first, end, stage0, count});
    const int64_t r0 = rec_begin(first), r1 = seg[4 * (size_t)(end - 1) + 2];
    P.max_records = std::max<int>(P.max_records, (int)(r1 - r0));
    auto pos = [&](int q) { return q == end ? r1 : rec_begin(q); };
    int prev = first;
    for (int g = 0; g <= ng; ++g) {
      int q = g == 0 ? first : g == ng ? end
                     : nearest_boundary(first, end, r0 + (r1 - r0) * g / ng, pos);
      q = std::max(q, prev);
      P.split.push_back(q);
      if (g > 0) {
        if (prev < q)
          P.group.insert(P.group.end(), {prev, q, seg[4 * (size_t)prev + 1], seg[4 * (size_t)(q - 1) + 2]});
        else
          P.group.insert(P.group.end(), {0, 0, 0, 0});
      }
      prev = q;
    }
    weight.push_back((r1 - r0) + (int64_t)stage_weight * count);
    open = -1;
  };

  for (int s = 0; s < NS; ++s) {
    const int ubeg = (int)(P.unit.size() / 4);
    for (int q = sbeg[s]; q < sbeg[s + 1]; ++q) {
      const int32_t *d = seg + 4 * (size_t)q;
      if (d[1] < 0 || d[2] <= d[1] || d[2] > nrec || d[3] < 0) return fail();
      P.endslot[d[2] - 1] = d[3];
      int own = 0, add = 0;        // distinct rows of the segment; of them not yet in the unit
      for (int64_t e = d[1]; e < d[2]; ++e) {
        if (off[e] == padoff) continue;
        if (off[e] < 0 || off[e] % rowbytes) return fail();
        const int c = off[e] / rowbytes;
        if (c >= cols) return fail();
        if (seen[c] != q) {
          seen[c] = q;
          ++own;
          if (open < 0 || stamp[c] != open) ++add;
        }
      }
      if (own > cap || d[2] - d[1] > nzcap) return fail();
      if (open < 0 || count + add > cap || d[2] - rec_begin(first) > nzcap) {
        close_unit(q);
        open = (int)(P.unit.size() / 4);
        first = q;
        count = 0;
      }
      for (int64_t e = d[1]; e < d[2]; ++e) {
        if (off[e] == padoff) continue;
        const int c = off[e] / rowbytes;
        if (stamp[c] != open) {
          stamp[c] = open;
          slot[c] = count++;
          P.stage.push_back(c);
        }
        P.off[e] = slot[c] * rowbytes;
        ++P.nonzeros;
      }
    }
    close_unit(sbeg[s + 1]);
    // workgroup ranges of this slice's units
    const int uend = (int)(P.unit.size() / 4);
    std::vector<int64_t> pre(uend - ubeg + 1, 0);
    for (int u = ubeg; u < uend; ++u) pre[u - ubeg + 1] = pre[u - ubeg] + weight[u];
    auto wpos = [&](int u) { return pre[u - ubeg]; };
    int prev = ubeg;
    for (int j = 0; j <= nbw; ++j) {
      int u = j == 0 ? ubeg : j == nbw ? uend
                     : nearest_boundary(ubeg, uend, pre.back() * j / nbw, wpos);
      u = std::max(u, prev);
      P.upart.push_back(u);
      prev = u;
    }
  }
  P.staged = 0;
  for (size_t u = 0; u < P.unit.size() / 4; ++u) P.staged += P.unit[4 * u + 3];
  return true;
}

// Tables the kernel reads: meta[2 u .. 2 u + 1] = (first record, records) of
// unit u; grp[2 (u ng + g) ..] = record range of lane group g relative to the
// unit's first record, (0, 0) for an empty range.
inline void unit_tables(const UnitPlan &P, const int32_t *seg, int ng, std::vector<int32_t> &meta,
                        std::vector<int32_t> &grp) {
  const size_t nunit = P.unit.size() / 4;
  meta.assign(2 * nunit, 0);
  grp.assign(2 * nunit * (size_t)ng, 0);
  for (size_t u = 0; u < nunit; ++u) {
    const int32_t r0 = seg[4 * (size_t)P.unit[4 * u] + 1];
    const int32_t r1 = seg[4 * (size_t)(P.unit[4 * u + 1] - 1) + 2];
    meta[2 * u] = r0;
    meta[2 * u + 1] = r1 - r0;
    for (int g = 0; g < ng; ++g) {
      const int32_t *d = &P.group[4 * (u * ng + g)];
      if (d[0] < d[1]) {
        grp[2 * (u * ng + g)] = d[2] - r0;
        grp[2 * (u * ng + g) + 1] = d[3] - r0;
      }
    }
  }
}

}  // namespace sfk
