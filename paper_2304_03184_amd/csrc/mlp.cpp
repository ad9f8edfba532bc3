// Network descriptor validation and layer layout.
#include "mlp_dev.hpp"

namespace nvr {

nvr_status build_net(const nvr_mlp_desc *m, Net *net) {
    NVR_REQUIRE(m != nullptr, NVR_EINVAL, "mlp descriptor is NULL");
    NVR_REQUIRE(m->n_in >= 1 && m->n_in <= 64, NVR_EINVAL, "n_in out of 1..64");
    NVR_REQUIRE(m->n_density_hidden >= 1 && m->n_density_hidden <= 4, NVR_EINVAL,
                "n_density_hidden out of 1..4");
    NVR_REQUIRE(m->n_colour_hidden >= 1 && m->n_colour_hidden <= 4, NVR_EINVAL,
                "n_colour_hidden out of 1..4");
    NVR_REQUIRE(m->density_out >= 1 && m->density_out <= 16, NVR_EINVAL, "density_out out of 1..16");
    NVR_REQUIRE(m->sh_degree >= 1 && m->sh_degree <= 4, NVR_EINVAL, "sh_degree out of 1..4");
    Net n{};
    n.n_in = m->n_in;
    n.dout = m->density_out;
    n.sh_degree = m->sh_degree;
    n.n_sh = m->sh_degree * m->sh_degree;
    int w = m->n_in, k = 0;
    for (int i = 0; i < m->n_density_hidden; ++i) {
        NVR_REQUIRE(m->density_hidden[i] >= 1 && m->density_hidden[i] <= 64, NVR_EINVAL,
                    "density width out of 1..64");
        n.in[k] = w;
        n.out[k] = m->density_hidden[i];
        w = n.out[k++];
    }
    n.in[k] = w;
    n.out[k++] = m->density_out;
    n.n_density = k;
    w = m->density_out + n.n_sh;
    NVR_REQUIRE(w <= 64, NVR_EINVAL, "colour input wider than 64");
    for (int i = 0; i < m->n_colour_hidden; ++i) {
        NVR_REQUIRE(m->colour_hidden[i] >= 1 && m->colour_hidden[i] <= 64, NVR_EINVAL,
                    "colour width out of 1..64");
        n.in[k] = w;
        n.out[k] = m->colour_hidden[i];
        w = n.out[k++];
    }
    n.in[k] = w;
    n.out[k++] = 3;
    n.n_layers = k;
    n.woff[0] = 0;
    for (int i = 0; i < k; ++i) n.woff[i + 1] = n.woff[i] + (int64_t)n.in[i] * n.out[i];
    *net = n;
    return NVR_OK;
}

}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_mlp_param_count(const nvr_mlp_desc *m, int64_t *count) {
    clear_error();
    NVR_REQUIRE(count != nullptr, NVR_EINVAL, "count is NULL");
    Net net;
    NVR_TRY(build_net(m, &net));
    *count = net.woff[net.n_layers];
    return NVR_OK;
}
