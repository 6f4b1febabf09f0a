// Autotuner cache: per-device-architecture choices of kernel variants, keyed
// by kernel and size bucket, kept in memory and in a small JSON file
// (ABDDC_TUNE_CACHE names the file; default $HOME/.cache/abddc/tune.json;
// "off" keeps the choices in memory only).
#pragma once

#include <string>

namespace abddc {

std::string device_arch(int device);
int tune_lookup(const std::string& key);          // -1 when the key is unknown
void tune_store(const std::string& key, int value);
// ceil(log2(max(v, 1))): the size bucket of a dimension
int size_bucket(long long v);

}  // namespace abddc
