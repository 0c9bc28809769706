// Host-side logic of the tvspec library (see host_logic.h).
#include "host_logic.h"

#include <cmath>

namespace tvspec {

thread_local std::string g_last_error;

static int validate_edges(const int *edges, int nb, int K)
{
    if (nb < 1 || nb > K)
        return fail(TVSPEC_EINVAL, "n_bands must be in [1, K]");
    if (edges[0] != 0 || edges[nb] != K)
        return fail(TVSPEC_EINVAL, "band edges must start at 0 and end at K");
    for (int j = 1; j <= nb; ++j)
        if (edges[j] <= edges[j - 1])
            return fail(TVSPEC_EINVAL, "band edges must be strictly increasing");
    return TVSPEC_OK;
}

int validate_shape(int B, int H, int W, int C, int iters)
{
    if (B < 1)
        return fail(TVSPEC_EINVAL, "B must be >= 1");
    if (H < 2 || W < 2)
        return fail(TVSPEC_EINVAL, "H and W must be >= 2");
    if (C < 1)
        return fail(TVSPEC_EINVAL, "C must be >= 1");
    if ((long long)B * C > 65535)
        return fail(TVSPEC_EINVAL, "B*C must be <= 65535");
    if ((long long)H * (long long)W > (1LL << 30))
        return fail(TVSPEC_EINVAL, "H*W must be <= 2^30");
    if ((long long)H * W * C * B > (1LL << 40))
        return fail(TVSPEC_EINVAL, "B*C*H*W too large");
    if (iters < 1)
        return fail(TVSPEC_EINVAL, "inner_iters must be >= 1");
    return TVSPEC_OK;
}

int validate_image(double dt, int K, const int *edges, int nb)
{
    if (!std::isfinite(dt) || !(dt > 0.0))
        return fail(TVSPEC_EINVAL, "dt must be finite and > 0");
    if (K < 1)
        return fail(TVSPEC_EINVAL, "K must be >= 1");
    return validate_edges(edges, nb, K);
}

int validate_opts(double tau, int warm, int precision, int ipl)
{
    if (!std::isfinite(tau) || !(tau > 0.0) || tau > 0.25)
        return fail(TVSPEC_EINVAL, "tau must be in (0, 0.25]");
    if (warm != 0 && warm != 1)
        return fail(TVSPEC_EINVAL, "warm_start must be 0 or 1");
    if (precision != TVSPEC_PRECISION_F32 && precision != TVSPEC_PRECISION_F64 &&
        precision != TVSPEC_PRECISION_MIXED)
        return fail(TVSPEC_EINVAL, "precision must be TVSPEC_PRECISION_F32, _F64 or _MIXED");
    const int maxt = precision == TVSPEC_PRECISION_F32 ? 16 : 8;
    if (ipl < 0 || ipl > maxt)
        return fail(TVSPEC_EINVAL, "iters_per_launch out of range");
    return TVSPEC_OK;
}

int validate_tile_shape(int tile_shape, int solver, int ipl)
{
    if (tile_shape != TVSPEC_TILE_SQUARE && tile_shape != TVSPEC_TILE_NARROW)
        return fail(TVSPEC_EINVAL, "tile_shape must be TVSPEC_TILE_SQUARE or TVSPEC_TILE_NARROW");
    if (tile_shape == TVSPEC_TILE_NARROW && solver != TVSPEC_SOLVER_CHAMBOLLE)
        return fail(TVSPEC_EINVAL, "the narrow tile shape is for the Chambolle solver");
    if (tile_shape == TVSPEC_TILE_NARROW && ipl > 8)
        return fail(TVSPEC_EINVAL, "the narrow tile shape takes iters_per_launch <= 8");
    return TVSPEC_OK;
}

void band_rows_of(const int *edges, int nbands, int *rows)
{
    rows[0] = 0; // sample 0 carries no phi
    for (int j = 0; j < nbands; ++j)
        for (int k = edges[j] + 1; k <= edges[j + 1]; ++k)
            rows[k] = j;
}

} // namespace tvspec
