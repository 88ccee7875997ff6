// Host access to the sparsity tables of gks_pattern.h.
#include "gks_pattern.h"

namespace gks {

const Pattern &pattern_tm()
{
    static const Pattern p{TM_N0, TM_NE, TM_NH, TM_R0, TM_C0, TM_RE, TM_CE, TM_RH, TM_CH};
    return p;
}
const Pattern &pattern_em()
{
    static const Pattern p{EM_N0, EM_NE, EM_NH, EM_R0, EM_C0, EM_RE, EM_CE, EM_RH, EM_CH};
    return p;
}

}  // namespace gks
