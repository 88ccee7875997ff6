// Host access to the sparsity tables of gks_pattern.h.
#include "gks_pattern.h"

namespace gks {

template <typename P>
static const Pattern &make()
{
    static const Pattern p{P::N0, P::NE, P::NH, P::R0, P::C0, P::RE, P::CE, P::RH, P::CH};
    return p;
}

const Pattern &pattern_cart(int model, int axis)
{
    if (model == GKS_TM2D) return axis == 0 ? make<PatTMx>() : make<PatTMy>();
    if (model == GKS_TM2D_PHM) return axis == 0 ? make<PatTPx>() : make<PatTPy>();
    if (model == GKS_EM3D_PHM) return axis == 0 ? make<PatEPx>() : (axis == 1 ? make<PatEPy>() : make<PatEPz>());
    return axis == 0 ? make<PatEMx>() : (axis == 1 ? make<PatEMy>() : make<PatEMz>());
}

const Pattern &pattern_cart_em_folded(int axis)
{
    return axis == 0 ? make<PatEMxF>() : (axis == 1 ? make<PatEMyF>() : make<PatEMzF>());
}

const Pattern &pattern_tet() { return make<PatTet>(); }

const Pattern &pattern_tri(int model) { return model == GKS_TM2D_PHM ? make<PatTriP>() : make<PatTri>(); }

}  // namespace gks
