"""More host-side checks of the C-ABI (no GPU needed)."""
from paper_2308_06484_amd import kdt as K


def test_graph_and_launch_calls_reject_null_context():
    L = K.lib()
    assert L.kdt_set_launch(None, 4) == K.E_ARG
    assert L.kdt_graph_launch(None, None) == K.E_ARG
    L.kdt_graph_destroy(None)
