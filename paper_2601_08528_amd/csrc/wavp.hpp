// Predictive replacement of workload-aware vector placement (Sec. 4.3,
// Alg. 2) over a full cache of C slots, for the placements of one batch.
//
// Alg. 2 takes F_min, the least F_lambda over residents whose reference bit
// is clear, then walks the clock hand: a slot with a set bit has it cleared,
// and the first slot with a clear bit holding F_min is replaced; the hand
// stays on it.  When every bit is set there is no F_min; the walk then goes
// round once clearing every bit, and F_min is taken over all residents.
//
// Within one batch the prediction of every resident is fixed, so the slots
// are scored once when the batch first needs a victim: f[s], the reference
// bits as one 64-bit mask per block of 64 slots, and per block the least f
// over its clear-bit slots, with a min tree over the blocks and a bitmap of
// the blocks that hold set bits (and over it, a bitmap of its nonzero words).
// An eviction then costs O(log C) plus the set bits its walk clears, instead
// of a pass over every slot.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <thread>
#include <vector>

namespace svf {

class WavpSweep {
 public:
  // Score all C slots: f_of(s) gives F_lambda of slot s's vector (every slot
  // is occupied), ref[s] its reference bit.  Runs on up to `threads` host
  // threads.  prefetch(s) is called kAhead slots before f_of(s), to request
  // the per-vector data f_of(s) will read (scattered over all vectors, it
  // would otherwise be one cache miss after another).
  template <class F, class P>
  void begin(int64_t C, F f_of, P prefetch, const uint8_t* ref, int threads) {
    C_ = C;
    nb_ = (C + 63) / 64;
    f_.resize(C);
    mask_.assign(nb_, 0);
    bmin_.resize(nb_);
    nw_ = (nb_ + 63) / 64;
    busy_.assign(nw_, 0);
    busy2_.assign((nw_ + 63) / 64, 0);
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(threads, nb_ / 512));
    auto work = [&](int t) {
      const int64_t b0 = nb_ * t / nt, b1 = nb_ * (t + 1) / nt;
      for (int64_t b = b0; b < b1; ++b) {
        uint64_t m = 0;
        double mn = kInf;
        const int64_t s1 = std::min(C, (b + 1) * 64);
        const int64_t pf_end = std::min(C, b1 * 64);
        for (int64_t s = b * 64; s < s1; ++s) {
          if (s + kAhead < pf_end) prefetch(s + kAhead);
          const double v = f_of(s);
          f_[s] = v;
          if (ref[s]) m |= 1ull << (s - b * 64);
          else if (v < mn) mn = v;
        }
        mask_[b] = m;
        bmin_[b] = mn;
      }
    };
    if (nt == 1) {
      work(0);
    } else {
      std::vector<std::thread> pool;
      for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
      work(0);
      for (auto& th : pool) th.join();
    }
    for (int64_t b = 0; b < nb_; ++b)
      if (mask_[b]) busy_[b >> 6] |= 1ull << (b & 63);
    for (int64_t w = 0; w < nw_; ++w)
      if (busy_[w]) busy2_[w >> 6] |= 1ull << (w & 63);
    P_ = 1;
    while (P_ < nb_) P_ <<= 1;
    tree_.assign(2 * P_, kInf);
    for (int64_t b = 0; b < nb_; ++b) tree_[P_ + b] = bmin_[b];
    for (int64_t i = P_ - 1; i >= 1; --i) tree_[i] = std::min(tree_[2 * i], tree_[2 * i + 1]);
    active_ = true;
  }
  bool active() const { return active_; }
  void end() { active_ = false; }

  // The slot Alg. 2 evicts with the hand at `clock`; clears, in ref[] too,
  // the set bits the hand passes and leaves the hand on the victim.
  int64_t evict(int64_t& clock, uint8_t* ref) {
    double fmin = tree_[1];
    if (fmin == kInf) {                      // every bit set: one round clears them all
      for (int64_t b = 0; b < nb_; ++b) {
        const int64_t s1 = std::min(C_, (b + 1) * 64);
        double mn = kInf;
        for (int64_t s = b * 64; s < s1; ++s) {
          ref[s] = 0;
          mn = std::min(mn, f_[s]);
        }
        mask_[b] = 0;
        bmin_[b] = mn;
        tree_[P_ + b] = mn;
      }
      std::fill(busy_.begin(), busy_.end(), 0ull);
      std::fill(busy2_.begin(), busy2_.end(), 0ull);
      for (int64_t i = P_ - 1; i >= 1; --i) tree_[i] = std::min(tree_[2 * i], tree_[2 * i + 1]);
      fmin = tree_[1];
    }
    const int64_t v = find_victim(clock, fmin);
    clear_range(clock, v, ref);
    clock = v;
    return v;
  }

  // The victim slot now holds a vector of prediction fx with a clear bit.
  void place(int64_t s, double fx) {
    f_[s] = fx;
    refresh_block(s >> 6);
  }

 private:
  static constexpr double kInf = std::numeric_limits<double>::infinity();
  static constexpr int64_t kAhead = 32;
  int64_t C_ = 0, nb_ = 0, nw_ = 0, P_ = 1;
  bool active_ = false;
  std::vector<double> f_, bmin_, tree_;
  std::vector<uint64_t> mask_, busy_, busy2_;

  void set_leaf(int64_t b, double v) {
    bmin_[b] = v;
    int64_t i = P_ + b;
    tree_[i] = v;
    for (i >>= 1; i >= 1; i >>= 1) tree_[i] = std::min(tree_[2 * i], tree_[2 * i + 1]);
  }
  void refresh_block(int64_t b) {
    double mn = kInf;
    const int64_t s1 = std::min(C_, (b + 1) * 64);
    for (int64_t s = b * 64; s < s1; ++s)
      if (!((mask_[b] >> (s - b * 64)) & 1ull)) mn = std::min(mn, f_[s]);
    set_leaf(b, mn);
  }
  // First slot of block b at or after slot `from` (inside b) with a clear bit
  // holding fmin, or -1.
  int64_t scan_block(int64_t b, int64_t from, int64_t to, double fmin) const {
    for (int64_t s = from; s < to; ++s)
      if (!((mask_[b] >> (s - b * 64)) & 1ull) && f_[s] == fmin) return s;
    return -1;
  }
  // First block in [lo, hi) whose clear-bit minimum is fmin (the global
  // minimum, so "<= fmin" finds it), or -1.
  int64_t first_block(int64_t lo, int64_t hi, double fmin) const {
    return first_block_rec(1, 0, P_, lo, hi, fmin);
  }
  int64_t first_block_rec(int64_t node, int64_t nl, int64_t nr, int64_t lo, int64_t hi,
                          double fmin) const {
    if (nr <= lo || hi <= nl || tree_[node] > fmin) return -1;
    if (nr - nl == 1) return nl;
    const int64_t mid = (nl + nr) / 2;
    const int64_t r = first_block_rec(2 * node, nl, mid, lo, hi, fmin);
    return r >= 0 ? r : first_block_rec(2 * node + 1, mid, nr, lo, hi, fmin);
  }
  int64_t find_victim(int64_t clock, double fmin) const {
    const int64_t b0 = clock >> 6;
    const int64_t end0 = std::min(C_, (b0 + 1) * 64);
    int64_t s = scan_block(b0, clock, end0, fmin);
    if (s >= 0) return s;
    int64_t b = first_block(b0 + 1, nb_, fmin);
    if (b < 0) b = first_block(0, b0, fmin);
    if (b >= 0) return scan_block(b, b * 64, std::min(C_, (b + 1) * 64), fmin);
    return scan_block(b0, b0 * 64, clock, fmin);   // only the slots before the hand remain
  }
  // Clear the set bits of the cyclic slot range [from, to).
  void clear_range(int64_t from, int64_t to, uint8_t* ref) {
    if (from == to) return;
    if (from < to) {
      clear_linear(from, to, ref);
    } else {
      clear_linear(from, C_, ref);
      clear_linear(0, to, ref);
    }
  }
  // First word index >= w0 of busy_ that is nonzero, or nw_.
  int64_t next_busy_word(int64_t w0) const {
    int64_t i = w0 >> 6;
    if (i >= (int64_t)busy2_.size()) return nw_;
    uint64_t m = busy2_[i] & (~0ull << (w0 & 63));
    while (m == 0) {
      if (++i >= (int64_t)busy2_.size()) return nw_;
      m = busy2_[i];
    }
    return i * 64 + __builtin_ctzll(m);
  }
  void clear_linear(int64_t from, int64_t to, uint8_t* ref) {
    if (from >= to) return;
    const int64_t bl = from >> 6, bh = (to - 1) >> 6;
    int64_t b = bl;
    while (b <= bh) {
      // skip blocks without set bits, a bitmap word at a time, and runs of
      // empty words through the bitmap over the words
      const uint64_t w = busy_[b >> 6] >> (b & 63);
      if (w == 0) {
        b = next_busy_word((b >> 6) + 1) << 6;
        continue;
      }
      b += __builtin_ctzll(w);
      if (b > bh) break;
      const int64_t lo = std::max(from, b * 64), hi = std::min(to, (b + 1) * 64);
      uint64_t sel = mask_[b];
      const int sh = (int)(lo - b * 64), n = (int)(hi - lo);
      const uint64_t range = (n == 64 ? ~0ull : ((1ull << n) - 1)) << sh;
      sel &= range;
      if (sel) {
        double mn = bmin_[b];
        for (uint64_t m = sel; m; m &= m - 1) {
          const int64_t s = b * 64 + __builtin_ctzll(m);
          ref[s] = 0;
          mn = std::min(mn, f_[s]);
        }
        mask_[b] &= ~sel;
        if (!mask_[b]) {
          busy_[b >> 6] &= ~(1ull << (b & 63));
          if (!busy_[b >> 6]) busy2_[b >> 12] &= ~(1ull << ((b >> 6) & 63));
        }
        set_leaf(b, mn);
      }
      ++b;
    }
  }
};

}  // namespace svf
