// kk_host.hpp -- host helpers shared by the libkk C-ABI translation units.
#pragma once
#include <stdarg.h>
#include <stdint.h>

#include <string>

#include "../../include/kk.h"
#include "kk_kernels.hpp"

namespace kk {

struct TileConfig {
  bool cyclic = false;  // one tile = whole lattice, wrapping inside LDS
  int tww = 8;          // interior words per tile row
  int th = 256;         // interior rows per tile
  int ku = 2;           // (row pair, word) units per thread
};

kk_status set_error(kk_status st, const char* fmt, ...);
void acceptance_table(double omega, uint64_t T[7], Accept* acc);
uint64_t place_count(int L, double composition);
int max_threads(int ku);
bool cyclic_fits(int L);
void default_tile(int L, int layout, TileConfig* tc);
int tile_geometry(int L, const TileConfig& tc, SweepParams* p);
bool tile_valid(int L, const TileConfig& tc, std::string* why);

}  // namespace kk
