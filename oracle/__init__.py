"""CPU oracle for per-edge typed graphlet counts (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package.  It is independent of the GPU library: no shared sources,
headers or tables.  See ``tg_oracle.c`` for what is computed and from which
parts of the paper.
"""

from .oracle import (  # noqa: F401
    build_oracle,
    row_width,
    global_width,
    pair_index,
    edge_row,
    edge_rows,
    all_edge_rows,
    global_counts,
    column_names,
    PA_BLOCKS,
    pa_row_width,
    pa_global_width,
    pa_column_names,
    pa_edge_rows,
    pa_all_edge_rows,
    pa_global_counts,
    pa_global_describe,
)
from .embedding import (  # noqa: F401
    graphlet_edge_weights,
    components,
    laplacian_spectrum,
    embedding,
)
from . import directed  # noqa: F401,E402
