"""Small scene builders shared by the tests (inputs only, no method arithmetic)."""
import numpy as np

import scenegen as sg


def scene_from_meshes(meshes, xforms=None, blas_id=None, mats=None, inst_mat=None,
                      camera=None, light=None, width=1, height=1, max_depth=1, mode=0, seed=0):
    n_inst = len(meshes) if xforms is None else len(xforms)
    if xforms is None:
        xforms = sg.identity_xform(n_inst)
    if blas_id is None:
        blas_id = np.arange(n_inst, dtype=np.uint32)
    if mats is None:
        mats = sg.materials([(sg.DIFFUSE, (0.8, 0.8, 0.8), 1.5)])
    if inst_mat is None:
        inst_mat = np.zeros(n_inst, np.uint32)
    if camera is None:
        camera = sg.Camera((0.0, 0.0, 5.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0)
    if light is None:
        light = sg.Light((0.0, 0.0, 10.0))
    return sg.Scene("test", list(meshes), np.asarray(xforms, np.float32).reshape(-1, 3, 4),
                    np.asarray(blas_id, np.uint32), np.asarray(inst_mat, np.uint32), mats,
                    camera, light, width, height, max_depth, mode, seed)


def tri_scene(tris, **kw):
    return scene_from_meshes([sg.triangles_mesh(tris)], **kw)


def ray(o, d, tmin=0.0, tmax=np.inf):
    return np.array(list(o) + list(d) + [tmin, tmax], np.float32)


def quad(z, half=2.0, normal_sign=1.0):
    """Square at height z in the xy-plane; winding normal along +z (or -z)."""
    a, b, c, d = (-half, -half, z), (half, -half, z), (half, half, z), (-half, half, z)
    if normal_sign > 0:
        return [(a, b, c), (a, c, d)]
    return [(a, c, b), (a, d, c)]
