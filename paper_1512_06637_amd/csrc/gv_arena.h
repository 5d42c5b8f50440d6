// FIFO ring allocator over the byte range [0, cap) of a memory arena (host
// code only, no GPU calls).  The serving engine keeps basket inputs and outputs
// in two such rings, one over a device arena and its pinned host mirror each.
//
// Blocks are carved at the head in allocation order, so baskets admitted one
// after another lie next to each other and a round of them moves with one copy
// per contiguous run.  Blocks may be released in any order; the space of a
// released block is reused once every older block is released too (the tail
// advances over the released prefix).  A block never wraps: when the space
// before the end is too short, that space becomes a dead pad and the block
// starts at offset 0.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <deque>

namespace gv {

class RingAlloc {
 public:
  static constexpr size_t npos = (size_t)-1;
  static constexpr size_t kAlign = 256;

  explicit RingAlloc(size_t cap = 0) : cap_(cap / kAlign * kAlign) {}

  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_; }  // bytes of live, released-but-held and pad blocks
  size_t blocks() const { return q_.size(); }
  static size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

  // Offset of a new block of `len` bytes (rounded up to kAlign), or npos if
  // there is no contiguous space now.  len == 0 or len > capacity(): npos.
  size_t alloc(size_t len) {
    len = round_up(len);
    if (len == 0 || len > cap_) return npos;
    if (q_.empty()) {
      head_ = 0;
      return place(0, len);
    }
    const size_t tail = q_.front().off;
    if (head_ > tail) {
      // free: [head, cap) and [0, tail)
      if (cap_ - head_ >= len) return place(head_, len);
      if (tail >= len) {
        if (head_ < cap_) push(head_, cap_ - head_, false);  // dead pad to the end
        return place(0, len);
      }
      return npos;
    }
    if (head_ < tail && tail - head_ >= len) return place(head_, len);
    return npos;  // head == tail with blocks held: full
  }

  // Releases the block that starts at `off` (must be live).  Returns false if
  // no live block starts there.
  bool release(size_t off) {
    bool found = false;
    for (auto& b : q_) {
      if (b.live && b.off == off) {
        b.live = false;
        found = true;
        break;
      }
    }
    while (!q_.empty() && !q_.front().live) {
      used_ -= q_.front().len;
      q_.pop_front();
    }
    if (q_.empty()) head_ = 0;
    return found;
  }

 private:
  struct Blk {
    size_t off, len;
    bool live;
  };
  size_t place(size_t off, size_t len) {
    push(off, len, true);
    head_ = off + len;  // may equal cap_; the next alloc then wraps or finds [cap, tail) empty
    return off;
  }
  void push(size_t off, size_t len, bool live) {
    q_.push_back(Blk{off, len, live});
    used_ += len;
  }
  size_t cap_, head_ = 0, used_ = 0;
  std::deque<Blk> q_;
};

}  // namespace gv
