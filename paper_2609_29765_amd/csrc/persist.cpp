// persist.cpp -- the analysed state (symbolic analysis, execution plan and
// reverse-mode plan) written to and read back from a byte stream, so that
// the once-per-pattern analysis, the dominant one-off cost (Sec. 6.6,
// Table 6), is paid once across processes.
//
// One field list per structure serves both directions: the writer and the
// reader visit the same fields in the same order, so they cannot drift
// apart.  Integers and doubles are stored as their host bytes (the stream is
// meant for the same library build on the same kind of host), vectors as a
// 64-bit length followed by their elements.  A header carries a magic, a
// format version and the sizes of the scalar types; the reader rejects a
// stream whose header, lengths or trailing checksum do not match.
#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/stc.h"
#include "analyse.hpp"

namespace stc {
namespace {

constexpr char kMagic[8] = {'S', 'T', 'C', 'P', 'L', 'A', 'N', '\0'};
constexpr uint32_t kVersion = 4;

// running checksum over a field's bytes: 64-bit words, then the tail
uint64_t mix(uint64_t h, const char* c, size_t n) {
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    std::memcpy(&w, c + i, 8);
    h = (h ^ w) * 0x100000001b3ull + (h >> 29);
  }
  for (; i < n; ++i) h = (h ^ (unsigned char)c[i]) * 0x100000001b3ull + 1;
  return h + n;
}

template <class A>
void fields(A& a, TileInfo& t) {
  a(t.m); a(t.k); a(t.cnt); a(t.true_cnt); a(t.contig); a(t.roff);
}

template <class A>
void fields(A& a, Symbolic& s) {
  a(s.n); a(s.qnz); a(s.qp); a(s.qi); a(s.perm); a(s.iperm); a(s.ndense); a(s.method); a(s.parent);
  a(s.lp); a(s.li); a(s.lnz); a(s.nb); a(s.NT); a(s.mode); a(s.route); a(s.tiles); a(s.rows); a(s.kd);
  a(s.phi); a(s.rho); a(s.sigma); a(s.tact); a(s.tasks); a(s.align); a(s.npad); a(s.pos);
}

template <class A>
void fields(A& a, Contrib& c) {
  a(c.a_off); a(c.b_off); a(c.a_rows); a(c.b_rows); a(c.rowmap); a(c.colmap);
}

template <class A>
void fields(A& a, UpdTask& u) {
  a(u.c_off); a(u.c_rows); a(u.diag); a(u.c_begin); a(u.c_end); a(u.level); a(u.big); a(u.partner);
  a(u.nsplit); a(u.part_off); a(u.in_part_off); a(u.in_npart);
}

template <class A>
void fields(A& a, TrsmTask& t) {
  a(t.x_off); a(t.l_off); a(t.rows); a(t.k);
}

template <class A>
void fields(A& a, Level& l) {
  a(l.big_items); a(l.upd_items); a(l.big_last); a(l.upd_last); a(l.potrf); a(l.trsm_items); a(l.flops);
  a(l.flops_potrf); a(l.flops_upd); a(l.flops_trsm);
}

template <class A>
void fields(A& a, Plan& p) {
  a(p.nb); a(p.NT); a(p.wg_slots); a(p.max_split); a(p.fold_pct); a(p.bm); a(p.parts); a(p.br); a(p.store); a(p.tile_off); a(p.vmap);
  a(p.maps); a(p.diag_h); a(p.tile_imap); a(p.contribs); a(p.upd); a(p.trsm); a(p.levels);
  a(p.row_tiles_ptr); a(p.row_tiles); a(p.col_tiles_ptr); a(p.col_tiles); a(p.fwd_level_ptr);
  a(p.fwd_level_blk); a(p.bwd_level_ptr); a(p.bwd_level_blk); a(p.flops_tile); a(p.flops_update);
  a(p.flops_potrf); a(p.flops_trsm); a(p.flops_exact); a(p.bytes_update);
}

template <class A>
void fields(A& a, ConTerm& c) {
  a(c.a_off); a(c.b_off); a(c.a_buf); a(c.a_mode); a(c.a_rmap); a(c.a_qmap); a(c.b_buf); a(c.b_qmap); a(c.K);
}

template <class A>
void fields(A& a, ConTask& t) {
  a(t.c_off); a(t.c_buf); a(t.c_rows); a(t.ncols); a(t.diag); a(t.t_begin); a(t.t_end); a(t.beta); a(t.alpha);
}

template <class A>
void fields(A& a, FoldTask& f) {
  a(f.c_off); a(f.c_buf); a(f.c_rows); a(f.ncols); a(f.diag); a(f.slot_off); a(f.nslots);
}

template <class A>
void fields(A& a, BackPlan& b) {
  a(b.terms); a(b.tasks); a(b.level_items); a(b.trtri_items); a(b.diagflag); a(b.folds); a(b.fold_items);
  a(b.slots); a(b.flops);
}

struct Writer {
  std::vector<char>* out;
  uint64_t sum = 0;
  void raw(const void* p, size_t n) {
    const char* c = static_cast<const char*>(p);
    sum = mix(sum, c, n);
    out->insert(out->end(), c, c + n);
  }
  template <class T>
  void operator()(T& v) {
    if constexpr (std::is_arithmetic_v<T>) {
      raw(&v, sizeof(T));
    } else {
      fields(*this, v);
    }
  }
  template <class T>
  void operator()(std::vector<T>& v) {
    uint64_t n = v.size();
    raw(&n, sizeof(n));
    if constexpr (std::is_arithmetic_v<T>) {
      if (n) raw(v.data(), sizeof(T) * n);
    } else {
      for (T& e : v) (*this)(e);
    }
  }
};

struct Reader {
  const char* p;
  size_t left;
  uint64_t sum = 0;
  bool ok = true;
  void raw(void* dst, size_t n) {
    if (!ok || n > left) {
      ok = false;
      return;
    }
    std::memcpy(dst, p, n);
    sum = mix(sum, p, n);
    p += n;
    left -= n;
  }
  template <class T>
  void operator()(T& v) {
    if constexpr (std::is_arithmetic_v<T>) {
      raw(&v, sizeof(T));
    } else {
      fields(*this, v);
    }
  }
  template <class T>
  void operator()(std::vector<T>& v) {
    uint64_t n = 0;
    raw(&n, sizeof(n));
    // a length beyond what is left cannot be real (each element takes at least a byte)
    if (!ok || n > left) {
      ok = false;
      return;
    }
    v.resize((size_t)n);
    if constexpr (std::is_arithmetic_v<T>) {
      if (n) raw(v.data(), sizeof(T) * n);
    } else {
      for (T& e : v) {
        (*this)(e);
        if (!ok) return;
      }
    }
  }
};

template <class A>
void header(A& a, uint32_t* version, uint32_t* sizes) {
  a(*version);
  for (int i = 0; i < 4; ++i) a(sizes[i]);
}

}  // namespace

int serialize_plan(Symbolic& s, Plan& p, BackPlan& b, std::vector<char>* out) {
  out->clear();
  out->insert(out->end(), kMagic, kMagic + sizeof(kMagic));
  Writer w{out};
  uint32_t version = kVersion;
  uint32_t sizes[4] = {sizeof(int32_t), sizeof(int64_t), sizeof(double), sizeof(size_t)};
  header(w, &version, sizes);
  w(s);
  w(p);
  w(b);
  const uint64_t sum = w.sum;
  out->insert(out->end(), reinterpret_cast<const char*>(&sum), reinterpret_cast<const char*>(&sum) + sizeof(sum));
  return 0;
}

int deserialize_plan(const char* data, size_t bytes, Symbolic* s, Plan* p, BackPlan* b, std::string* why) {
  if (bytes < sizeof(kMagic) + sizeof(uint64_t) || std::memcmp(data, kMagic, sizeof(kMagic)) != 0) {
    *why = "not a saved stc analysis (bad magic)";
    return STC_ERR_ARG;
  }
  Reader r{data + sizeof(kMagic), bytes - sizeof(kMagic) - sizeof(uint64_t)};
  uint32_t version = 0, sizes[4] = {0, 0, 0, 0};
  header(r, &version, sizes);
  if (!r.ok || version != kVersion || sizes[0] != sizeof(int32_t) || sizes[1] != sizeof(int64_t) ||
      sizes[2] != sizeof(double) || sizes[3] != sizeof(size_t)) {
    *why = "saved analysis has another format version or type sizes";
    return STC_ERR_ARG;
  }
  r(*s);
  if (r.ok) r(*p);
  if (r.ok) r(*b);
  uint64_t sum = 0;
  std::memcpy(&sum, data + bytes - sizeof(sum), sizeof(sum));
  if (!r.ok || r.left != 0 || sum != r.sum) {
    *why = "saved analysis is truncated or corrupted";
    return STC_ERR_ARG;
  }
  build_lmap(*s, p);
  return 0;
}

}  // namespace stc
