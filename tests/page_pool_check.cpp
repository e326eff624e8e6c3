// Host-only unit check of the serving loop's page pool (page_pool.h): the
// memory cap, slab growth through the allocator callback, reuse of released
// pages, refusal without side effects.  Built with g++, no GPU involved.
#include <cstdio>
#include <set>
#include <vector>

#include "page_pool.h"

static int failures = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);            \
      ++failures;                                                 \
    }                                                             \
  } while (0)

int main() {
  using mg::PagePool;
  std::vector<std::pair<long, long>> slabs;
  bool refuse = false;
  PagePool pool(10, 4, [&](int64_t first, int64_t n) {
    if (refuse) return false;
    slabs.push_back({first, n});
    return true;
  });
  CHECK(PagePool::pages_for({0, 0}) == 0);
  CHECK(PagePool::pages_for({1, 64}) == 2);
  CHECK(PagePool::pages_for({65, 128, 3}) == 5);
  CHECK(pool.fits(10) && !pool.fits(11) && pool.ever_fits(10) && !pool.ever_fits(11));
  std::vector<int64_t> a, b, c;
  CHECK(pool.allocate(3, a) && a.size() == 3);
  CHECK(slabs.size() == 1 && slabs[0].first == 0 && slabs[0].second == 4);
  CHECK(pool.allocate(6, b) && b.size() == 6);               // second slab, then a partial one
  CHECK(pool.created_pages() == 10 && slabs.size() == 3 && slabs[2].second == 2);
  CHECK(!pool.allocate(2, c) && c.empty() && pool.used_pages() == 9);   // over the cap
  CHECK(pool.allocate(1, c) && c.size() == 1);
  std::set<int64_t> all(a.begin(), a.end());
  all.insert(b.begin(), b.end());
  all.insert(c.begin(), c.end());
  CHECK(all.size() == 10 && *all.begin() == 0 && *all.rbegin() == 9);  // distinct, in range
  pool.release(b);
  CHECK(pool.used_pages() == 4 && pool.fits(6) && !pool.fits(7));
  std::vector<int64_t> d;
  CHECK(pool.allocate(6, d) && pool.created_pages() == 10);            // reuse, no new slab
  std::set<int64_t> sb(b.begin(), b.end()), sd(d.begin(), d.end());
  CHECK(sb == sd);
  // a refusing allocator leaves the pool unchanged
  PagePool p2(8, 8, [&](int64_t, int64_t) { return false; });
  std::vector<int64_t> e;
  CHECK(!p2.allocate(1, e) && e.empty() && p2.used_pages() == 0 && p2.created_pages() == 0);
  // reserve creates slabs up front (at most up to the cap); allocations then reuse them
  std::vector<std::pair<long, long>> s3;
  PagePool p3(10, 4, [&](int64_t first, int64_t n) {
    s3.push_back({first, n});
    return true;
  });
  CHECK(p3.reserve(5) && p3.created_pages() == 8 && s3.size() == 2 && p3.used_pages() == 0);
  std::vector<int64_t> f;
  CHECK(p3.allocate(8, f) && s3.size() == 2);                         // no new slab
  CHECK(p3.reserve(100) && p3.created_pages() == 10 && s3.size() == 3);  // capped
  CHECK(p3.reserve(3) && s3.size() == 3);                              // nothing to add
  PagePool p4(8, 4, [&](int64_t, int64_t) { return false; });
  CHECK(!p4.reserve(4) && p4.created_pages() == 0);
  std::printf("page pool check: %d failures\n", failures);
  return failures ? 1 : 0;
}
