// FASTA ingest on the host's cores: header lines ('>' at a line start) start
// records, every other line holds bases; line breaks ("\n" or "\r\n") and
// blanks are dropped.  The records' bases are written back to back as bytes
// (the scans treat anything but A/C/G/T/a/c/g/t as a reset) or as 2-bit codes
// with a 1-bit N mask, ready to be copied to the device and scanned whole or
// record by record (coex_seq.first_base).  Bases before the first header
// line form a record of their own; a text without header lines is one record.
//
// The text is cut into pieces at line starts, one per worker thread.  A first
// pass counts each piece's bases, header lines and bases before its first
// header; prefix sums of those give every piece its first output position and
// its first record index; a second pass writes the bases and the record
// starts.  Record lengths follow from consecutive starts.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "coex.h"

namespace {

inline bool is_blank(uint8_t c) { return c == '\n' || c == '\r' || c == ' ' || c == '\t' || c == '\v' || c == '\f'; }
inline bool is_lower(uint8_t c) { return c >= 'a' && c <= 'z'; }

// 2-bit code of A/C/G/T (either case), or -1.
inline int code_of(uint8_t c) {
  switch (c | 0x20) {
    case 'a': return 0;
    case 'c': return 1;
    case 'g': return 2;
    case 't': return 3;
    default: return -1;
  }
}

struct Piece {
  uint64_t lo = 0, hi = 0;              // text bytes [lo, hi), lo at a line start
  uint64_t bases = 0, headers = 0;      // first pass
  uint64_t lead = 0;                    // bases before the piece's first header (all, if none)
  uint64_t out0 = 0, rec0 = 0, out1 = 0;  // output positions [out0, out1), index of its first header's record
};

// Walks text [lo, hi) line by line: base(byte) for every base, header(offset)
// at every header line.
template <class OnBase, class OnHeader>
void walk(const uint8_t* t, uint64_t lo, uint64_t hi, OnBase&& base, OnHeader&& header) {
  uint64_t i = lo;
  while (i < hi) {
    if (t[i] == '>') {
      header(i);
      const void* nl = std::memchr(t + i, '\n', hi - i);
      i = nl ? (uint64_t)(static_cast<const uint8_t*>(nl) - t) + 1 : hi;
      continue;
    }
    for (; i < hi && t[i] != '\n'; ++i)
      if (!is_blank(t[i])) base(t[i]);
    if (i < hi) ++i;
  }
}

std::vector<Piece> cut(const uint8_t* t, uint64_t len, uint32_t threads) {
  if (threads == 0) threads = std::max(1u, std::thread::hardware_concurrency());
  // pieces of at least 1 MiB: short texts are not worth a thread each
  const uint64_t step = std::max<uint64_t>(1ull << 20, (len + threads - 1) / threads);
  std::vector<Piece> ps;
  uint64_t lo = 0;
  while (lo < len) {
    uint64_t hi = std::min(len, lo + step);
    if (hi < len) {  // the cut moves to the next line start
      const void* nl = std::memchr(t + hi - 1, '\n', len - (hi - 1));
      hi = nl ? (uint64_t)(static_cast<const uint8_t*>(nl) - t) + 1 : len;
    }
    Piece p;
    p.lo = lo;
    p.hi = hi;
    ps.push_back(p);
    lo = hi;
  }
  return ps;
}

template <class F>
void parallel(std::vector<Piece>& ps, F&& f) {
  std::vector<std::thread> pool;
  for (size_t i = 1; i < ps.size(); ++i) pool.emplace_back([&, i]() { f(ps[i]); });
  if (!ps.empty()) f(ps[0]);
  for (auto& th : pool) th.join();
}

struct Layout {
  uint64_t records = 0, bases = 0;  // output bases, separators included
  bool leading = false;             // a record before the first header line
};

// First pass and prefix sums.
Layout plan(const uint8_t* t, uint64_t len, bool separate, std::vector<Piece>& ps) {
  parallel(ps, [&](Piece& p) {
    bool seen = false;
    walk(t, p.lo, p.hi,
         [&](uint8_t) {
           ++p.bases;
           if (!seen) ++p.lead;
         },
         [&](uint64_t) {
           ++p.headers;
           seen = true;
         });
  });
  Layout L;
  uint64_t headers = 0, before_first = 0;
  bool found = false;
  for (const Piece& p : ps) {
    if (!found) before_first += p.lead;
    if (p.headers) found = true;
    headers += p.headers;
  }
  L.leading = len > 0 && (before_first > 0 || headers == 0);
  L.records = headers + (L.leading ? 1 : 0);
  const uint64_t sep = separate ? 1 : 0;
  uint64_t out = 0, rec = L.leading ? 1 : 0;
  for (Piece& p : ps) {
    p.out0 = out;
    p.rec0 = rec;
    // a separator in front of every record but the first
    out += p.bases + sep * (rec == 0 && p.headers ? p.headers - 1 : p.headers);
    rec += p.headers;
    p.out1 = out;
  }
  L.bases = out;
  return L;
}

// 2-bit output of one piece: whole bytes it owns are stored, the bytes it
// shares with a neighbouring piece (its first and last) are OR-ed in.
struct Packer {
  uint8_t* codes;
  uint8_t* mask;
  uint64_t out0, out1;
  uint64_t pos;
  uint32_t cb = 0, mb = 0;  // code and mask bits of the byte being filled
  void flush_code(uint64_t byte) {
    const bool shared = (byte == out0 / 4 && (out0 & 3)) || (byte == (out1 - 1) / 4 && (out1 & 3));
    if (shared) __atomic_fetch_or(codes + byte, (uint8_t)cb, __ATOMIC_RELAXED);
    else codes[byte] = (uint8_t)cb;
    cb = 0;
  }
  void flush_mask(uint64_t byte) {
    if (!mask) { mb = 0; return; }
    const bool shared = (byte == out0 / 8 && (out0 & 7)) || (byte == (out1 - 1) / 8 && (out1 & 7));
    if (shared) __atomic_fetch_or(mask + byte, (uint8_t)mb, __ATOMIC_RELAXED);
    else mask[byte] = (uint8_t)mb;
    mb = 0;
  }
  void put(int code) {  // code < 0: N
    if (code < 0) mb |= 1u << (pos & 7);
    else cb |= (uint32_t)code << (2 * (pos & 3));
    ++pos;
    if ((pos & 3) == 0) flush_code((pos - 1) / 4);
    if ((pos & 7) == 0) flush_mask((pos - 1) / 8);
  }
  void finish() {
    if (pos & 3) flush_code(pos / 4);
    if (pos & 7) flush_mask(pos / 8);
  }
};

}  // namespace

extern "C" int coex_fasta_measure(const char* text, uint64_t len, uint32_t flags, uint32_t threads,
                                  uint64_t* n_records, uint64_t* n_bases) {
  if ((!text && len) || !n_records || !n_bases) return COEX_EINVAL;
  if (flags & ~(COEX_FASTA_SOFTMASK | COEX_FASTA_SEPARATE)) return COEX_EINVAL;
  try {
    const uint8_t* t = reinterpret_cast<const uint8_t*>(text);
    std::vector<Piece> ps = cut(t, len, threads);
    const Layout L = plan(t, len, flags & COEX_FASTA_SEPARATE, ps);
    *n_records = L.records;
    *n_bases = L.bases;
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

extern "C" int coex_fasta_read(const char* text, uint64_t len, int32_t encoding, uint32_t flags, uint32_t threads,
                               void* bases, uint8_t* n_mask, uint64_t cap_bases, uint64_t* rec_start,
                               uint64_t* rec_len, uint64_t* rec_header, uint64_t cap_records, uint64_t* n_records,
                               uint64_t* n_bases) {
  if ((!text && len) || !n_records || !n_bases) return COEX_EINVAL;
  if (flags & ~(COEX_FASTA_SOFTMASK | COEX_FASTA_SEPARATE)) return COEX_EINVAL;
  if (encoding != COEX_ENC_BYTE && encoding != COEX_ENC_2BIT) return COEX_EINVAL;
  try {
    const uint8_t* t = reinterpret_cast<const uint8_t*>(text);
    const bool soft = flags & COEX_FASTA_SOFTMASK;
    const bool separate = flags & COEX_FASTA_SEPARATE;
    std::vector<Piece> ps = cut(t, len, threads);
    const Layout L = plan(t, len, separate, ps);
    *n_records = L.records;
    *n_bases = L.bases;
    if (L.bases > cap_bases || ((rec_start || rec_len || rec_header) && L.records > cap_records))
      return COEX_ECAPACITY;
    if (L.bases && !bases) return COEX_EINVAL;
    if (encoding == COEX_ENC_2BIT) {
      // bytes that no piece fills whole are OR-ed into: start from zero
      std::memset(bases, 0, (L.bases + 3) / 4);
      if (n_mask) std::memset(n_mask, 0, (L.bases + 7) / 8);
    }
    if (L.leading) {
      if (rec_start) rec_start[0] = 0;
      if (rec_header) rec_header[0] = UINT64_MAX;
    }
    parallel(ps, [&](Piece& p) {
      uint64_t rec = p.rec0;
      if (encoding == COEX_ENC_BYTE) {
        uint8_t* out = static_cast<uint8_t*>(bases);
        uint64_t o = p.out0;
        walk(t, p.lo, p.hi, [&](uint8_t c) { out[o++] = soft && is_lower(c) ? (uint8_t)'N' : c; },
             [&](uint64_t at) {
               if (separate && rec > 0) out[o++] = 'N';
               if (rec_start) rec_start[rec] = o;
               if (rec_header) rec_header[rec] = at;
               ++rec;
             });
      } else {
        Packer pk{static_cast<uint8_t*>(bases), n_mask, p.out0, p.out1, p.out0};
        walk(t, p.lo, p.hi, [&](uint8_t c) { pk.put(soft && is_lower(c) ? -1 : code_of(c)); },
             [&](uint64_t at) {
               if (separate && rec > 0) pk.put(-1);
               if (rec_start) rec_start[rec] = pk.pos;
               if (rec_header) rec_header[rec] = at;
               ++rec;
             });
        pk.finish();
      }
    });
    if (rec_len) {
      std::vector<uint64_t> own;
      const uint64_t* st = rec_start;
      if (!st) {  // starts are needed for the lengths
        own.resize(L.records);
        uint64_t r = 0, o = 0;
        if (L.leading) own[r++] = 0;
        for (const Piece& p : ps) {
          o = p.out0;
          walk(t, p.lo, p.hi, [&](uint8_t) { ++o; }, [&](uint64_t) {
            if (separate && r > 0) ++o;
            own[r++] = o;
          });
        }
        st = own.data();
      }
      for (uint64_t r = 0; r < L.records; ++r)
        rec_len[r] = (r + 1 < L.records ? st[r + 1] - (separate ? 1 : 0) : L.bases) - st[r];
    }
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}
