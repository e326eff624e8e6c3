// page_pool.h -- host-only bookkeeping of the serving loop's device pages:
// memory-capped page allocation (slabs obtained through a callback) and the
// admission test.  No HIP calls here, so the logic is testable on the CPU.
//
// A page holds PAGE_ENVS environments of one vehicle class.  Pages live in
// slabs of slab_pages pages; a slab is requested from the allocator callback
// only when the free list is empty and the cap still allows it.  The cap is a
// number of pages derived from the memory budget (e.g. 80 % of HBM).
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace mg {

constexpr int kPageEnvs = 64;

class PagePool {
 public:
  // alloc_slab(first_page, n_pages) must make pages [first, first + n) usable
  // and return false if the memory could not be obtained.
  using SlabAlloc = std::function<bool(int64_t first_page, int64_t n_pages)>;

  PagePool(int64_t cap_pages, int64_t slab_pages, SlabAlloc alloc)
      : cap_(cap_pages), slab_(slab_pages > 0 ? slab_pages : 1), alloc_(std::move(alloc)) {}

  int64_t cap_pages() const { return cap_; }
  int64_t used_pages() const { return used_; }
  int64_t created_pages() const { return created_; }
  int64_t free_pages_within_cap() const { return cap_ - used_; }

  // Pages a request needs: one run of pages per class.
  static int64_t pages_for(const std::vector<int64_t>& per_class_envs) {
    int64_t n = 0;
    for (int64_t c : per_class_envs) n += (c + kPageEnvs - 1) / kPageEnvs;
    return n;
  }

  // Admission test: the request fits in the cap right now.
  bool fits(int64_t n_pages) const { return n_pages <= cap_ - used_; }
  // A request larger than the whole cap can never be admitted.
  bool ever_fits(int64_t n_pages) const { return n_pages <= cap_; }

  // Allocates n pages (ids appended to out); false (and no change) if the cap
  // or the slab allocator refuses.
  bool allocate(int64_t n, std::vector<int64_t>& out) {
    if (n < 0 || !fits(n)) return false;
    while ((int64_t)free_.size() < n)
      if (!add_slab()) return false;
    for (int64_t i = 0; i < n; ++i) {
      out.push_back(free_.back());
      free_.pop_back();
    }
    used_ += n;
    return true;
  }

  void release(const std::vector<int64_t>& pages) {
    for (int64_t p : pages) free_.push_back(p);
    used_ -= (int64_t)pages.size();
  }

  // Creates slabs up front until at least min(n_pages, cap) pages exist, so
  // that later allocations need no allocator call; false if the allocator
  // refuses (the slabs created so far stay).
  bool reserve(int64_t n_pages) {
    const int64_t want = n_pages < cap_ ? n_pages : cap_;
    while (created_ < want)
      if (!add_slab()) return false;
    return true;
  }

 private:
  bool add_slab() {
    const int64_t room = cap_ - created_;
    if (room <= 0) return false;
    const int64_t add = room < slab_ ? room : slab_;
    if (!alloc_(created_, add)) return false;
    for (int64_t p = created_ + add - 1; p >= created_; --p) free_.push_back(p);
    created_ += add;
    return true;
  }

  int64_t cap_, slab_;
  SlabAlloc alloc_;
  int64_t used_ = 0, created_ = 0;
  std::vector<int64_t> free_;
};

}  // namespace mg
