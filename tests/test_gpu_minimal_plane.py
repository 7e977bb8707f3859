"""Shadow gradients need the light-view edge smoothing: on the minimal-plane
scene a displaced occluder corner is recovered with it and stays put without
it, for any filter size; a displaced occluder is recovered with Adam."""
import pytest

pytestmark = pytest.mark.gpu


def test_corner_recovered_only_with_light_smoothing():
    from paper_2308_10896_amd import minimal_plane as mp
    for k in (1, 5):
        on = mp.vertex_experiment(k, True, iters=100)
        off = mp.vertex_experiment(k, False, iters=100)
        print('k', k, 'AA on', on['error_initial'], '->', on['error_final'],
              '| AA off', off['error_initial'], '->', off['error_final'], flush=True)
        assert on['error_final'] < 0.25 * on['error_initial']
        assert off['error_final'] > 0.9 * off['error_initial']


def test_translation_recovered():
    from paper_2308_10896_amd import minimal_plane as mp
    r = mp.translation_experiment(5, 'adam', 0.01, iters=100)
    e = r['signed_error']
    print('signed error', e[0], e[50], e[-1], flush=True)
    assert abs(e[-1]) < 0.2 * abs(e[0])
