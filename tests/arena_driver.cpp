// Host-only driver of rta::RowArena for tests/test_arena.py: reads commands
// from stdin and prints one result line per command.
//   c N    reset to capacity N       -> "ok"
//   a N    alloc N rows              -> start or -1
//   r S N  release [S, S+N)          -> 1 or 0
//   s      state                     -> "used largest start:len ..."
#include <cstdio>
#include <iostream>
#include <string>

#include "arena.hpp"

int main() {
  rta::RowArena ar;
  std::string cmd;
  while (std::cin >> cmd) {
    if (cmd == "c") {
      long long n;
      std::cin >> n;
      ar.reset(n);
      std::printf("ok\n");
    } else if (cmd == "a") {
      long long n;
      std::cin >> n;
      std::printf("%lld\n", (long long)ar.alloc(n));
    } else if (cmd == "r") {
      long long s, n;
      std::cin >> s >> n;
      std::printf("%d\n", ar.release(s, n) ? 1 : 0);
    } else if (cmd == "s") {
      std::printf("%lld %lld", (long long)ar.used(), (long long)ar.largest_free());
      for (const auto& f : ar.free_ranges()) std::printf(" %lld:%lld", (long long)f.first, (long long)f.second);
      std::printf("\n");
    }
  }
  return 0;
}
