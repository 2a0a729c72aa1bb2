// Autotuner cache of the batched plan: a JSON file holding, per key, the
// chosen shape of the Bluestein column path and its measured time.
//   {"version": 1, "entries": {"<key>": {"l1": 8, "mb": 16, "kb": 16,
//                                        "pchunk": 0, "fuse": 1, "nat": 0, "us": 1234.5}, ...}}
// The key names the device and the problem ("gfx950:256cu|f32|N4096|T4|m16").
// Host code only.
#pragma once
#include <map>
#include <string>

namespace ipfb {

struct TuneEntry {
  int l1 = 0, mb = 16, kb = 16, pchunk = 0, fuse = 1, nat = 0;  // fuse 1, nat 0 when the file has none
  double us = 0.0;
};

// Reads every entry of the file into out (entries already in out are kept
// unless the file has the same key). A missing file reads as empty and returns
// true; a file that does not parse returns false and leaves out unchanged.
bool tune_cache_read(const std::string& path, std::map<std::string, TuneEntry>& out);

// Writes the entries (the file's current entries merged with these, these
// winning) through a temporary file renamed over the path. false on I/O error.
bool tune_cache_write(const std::string& path, const std::map<std::string, TuneEntry>& entries);

}  // namespace ipfb
