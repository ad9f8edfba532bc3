// Layer bookkeeping of the density + colour networks (host side).
#pragma once
#include "common.hpp"

namespace nvr {

constexpr int kMaxLayers = 10;
constexpr float kSigmaClamp = 15.f;

struct Net {
    int n_layers;          // density layers, then colour layers
    int n_density;         // number of density layers
    int in[kMaxLayers], out[kMaxLayers];
    int64_t woff[kMaxLayers + 1];   // flat parameter offsets (woff[n_layers] = total)
    int n_in, dout, sh_degree, n_sh;
};

nvr_status build_net(const nvr_mlp_desc *m, Net *net);


}  // namespace nvr
