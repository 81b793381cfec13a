// Configuration space, features and knowledge-base keys shared by the
// auto-tuner and the cost model.
#pragma once
#include <string>
#include <vector>

#include "internal.h"

namespace skel {

constexpr int kNumFeatures = 24;

// Every valid configuration of a chain at a shape (tuner search space).
std::vector<Config> enumerate_configs(const Linear& L, const Shape& sh);
// The 24 cost-model features of (chain, shape, configuration).
void features(const Linear& L, const Shape& sh, const Config& c, float* f);
// Text key of a (chain, shape) pair in the tuning database.
std::string composition_key(const Linear& L, const Shape& sh);
void config_to_opts(const Config& c, skel_plan_opts* o);

}  // namespace skel
