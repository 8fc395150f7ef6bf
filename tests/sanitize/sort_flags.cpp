// The cell sort's integrity checks (pic_internal.h) and their report
// (setup.cpp), on the host: the same constexpr functions the sort kernels
// call decide which bits a tile, slot or source raises.
#include <cstdio>
#include <cstring>

#include "../../paper_2303_12874_amd/csrc/pic_internal.h"

using namespace pic;

static int fails = 0;
#define CHECK(c)                                       \
  do {                                                 \
    if (!(c)) {                                        \
      std::printf("FAILED %s:%d %s\n", __FILE__, __LINE__, #c); \
      ++fails;                                         \
    }                                                  \
  } while (0)

int main() {
  const long long np = 1000;
  // the counts' total must be the electron count
  CHECK(sort_count_flags(np, np) == 0);
  CHECK(sort_count_flags(np - 1, np) == kSortBadCount);
  CHECK(sort_count_flags(np + 1, np) == kSortBadCount);
  // a tile's range [beg, end) inside [0, np]; an empty tile is fine
  CHECK(sort_tile_flags(0, 0, np) == 0);
  CHECK(sort_tile_flags(10, 10, np) == 0);
  CHECK(sort_tile_flags(0, np, np) == 0);
  CHECK(sort_tile_flags(-1, 5, np) == kSortBadTile);
  CHECK(sort_tile_flags(5, np + 1, np) == kSortBadTile);
  CHECK(sort_tile_flags(7, 6, np) == kSortBadTile);
  // slots and sources in [0, np)
  CHECK(sort_index_flags(0, np, kSortBadSlot) == 0);
  CHECK(sort_index_flags(np - 1, np, kSortBadSource) == 0);
  CHECK(sort_index_flags(np, np, kSortBadSlot) == kSortBadSlot);
  CHECK(sort_index_flags(-3, np, kSortBadSource) == kSortBadSource);
  // distinct bits, so that raised ones combine
  CHECK((kSortBadCount | kSortBadTile | kSortBadSlot | kSortBadSource) == 15u);
  // the report names the run and every raised bit, and nothing when none is
  char buf[320];
  CHECK(sort_flags_text(0, 2, buf, sizeof buf) == 0 && buf[0] == 0);
  CHECK(sort_flags_text(kSortBadTile | kSortBadSource, 2, buf, sizeof buf) == (kSortBadTile | kSortBadSource));
  CHECK(std::strstr(buf, "run 2") && std::strstr(buf, "tile") && std::strstr(buf, "source"));
  CHECK(!std::strstr(buf, "sum") && !std::strstr(buf, "slot"));
  char tiny[8];  // a short buffer is never overrun
  sort_flags_text(15u, 0, tiny, sizeof tiny);
  CHECK(std::strlen(tiny) < sizeof tiny);
  if (fails) return 1;
  std::printf("sort flags ok\n");
  return 0;
}
