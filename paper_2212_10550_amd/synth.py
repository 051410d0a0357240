"""Seeded synthetic workloads for the articulated-NeRF deform-and-query path.

This module only *generates inputs*: skeletons, bone transforms, skinning
weight grids, occupancy masks, camera rays, hash tables, MLP weights and
target colours.  It contains none of the method's arithmetic (no skinning,
no root finding, no encoding, no compositing), so both the HIP path and the
FP64 oracle can consume its output without sharing any computation.

Every generator works in float64 and returns float64; ``Workload`` rounds
each array once to its storage dtype (float32 / float16 / uint8) and both
sides read exactly those rounded values.

The paper's own inputs (PeopleSnapshot video, SMPL, Anim-NeRF poses; Sec. 4.1)
are not available; these synthetic stand-ins have the same structure: a
24-bone human skeleton (the SMPL joint count used by the skinning field of
Sec. 3.1, Eq. 5-7), a low-resolution skinning-weight voxel grid, a binary
occupancy grid around the posed body (Sec. 3.3) and a 540x540 camera (the
render resolution quoted in Sec. 4.2).
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

NB = 24

# 24-joint humanoid tree in SMPL order: (name, parent, T-pose (x, y) offset
# relative to the pelvis in a unit-height figure).  The figure stands in the
# plane z = 0.5, head up (+y), facing -z (towards the camera).
_JOINTS = [
    ("pelvis", -1, (0.00, 0.00)),
    ("l_hip", 0, (0.07, -0.05)),
    ("r_hip", 0, (-0.07, -0.05)),
    ("spine1", 0, (0.00, 0.07)),
    ("l_knee", 1, (0.08, -0.22)),
    ("r_knee", 2, (-0.08, -0.22)),
    ("spine2", 3, (0.00, 0.14)),
    ("l_ankle", 4, (0.08, -0.39)),
    ("r_ankle", 5, (-0.08, -0.39)),
    ("spine3", 6, (0.00, 0.20)),
    ("l_foot", 7, (0.09, -0.43)),
    ("r_foot", 8, (-0.09, -0.43)),
    ("neck", 9, (0.00, 0.28)),
    ("l_collar", 9, (0.04, 0.25)),
    ("r_collar", 9, (-0.04, 0.25)),
    ("head", 12, (0.00, 0.35)),
    ("l_shoulder", 13, (0.10, 0.26)),
    ("r_shoulder", 14, (-0.10, 0.26)),
    ("l_elbow", 16, (0.21, 0.26)),
    ("r_elbow", 17, (-0.21, 0.26)),
    ("l_wrist", 18, (0.32, 0.26)),
    ("r_wrist", 19, (-0.32, 0.26)),
    ("l_hand", 20, (0.37, 0.26)),
    ("r_hand", 21, (-0.37, 0.26)),
]
# Segment end per joint: the child the bone points at (a leaf is a point).
_SEG_END = {0: 3, 1: 4, 2: 5, 3: 6, 4: 7, 5: 8, 6: 9, 7: 10, 8: 11, 9: 12,
            12: 15, 13: 16, 14: 17, 16: 18, 17: 19, 18: 20, 19: 21, 20: 22, 21: 23}


@dataclasses.dataclass(frozen=True)
class Skeleton:
    joints: np.ndarray   # [NB, 3] rest joint positions (canonical space)
    parents: np.ndarray  # [NB] parent index, -1 for the root
    seg_a: np.ndarray    # [NB, 3] bone segment start (= joint)
    seg_b: np.ndarray    # [NB, 3] bone segment end (first child, or the joint for leaves)


def make_skeleton(seed: int = 0) -> Skeleton:
    rng = np.random.default_rng(seed)
    centre = np.array([0.5, 0.52, 0.5])
    j = np.zeros((NB, 3))
    for i, (_, _, (ox, oy)) in enumerate(_JOINTS):
        j[i] = centre + np.array([ox, oy, 0.0])
    j += rng.normal(0.0, 0.01, size=j.shape)
    j = np.clip(j, 0.05, 0.95)
    parents = np.array([p for _, p, _ in _JOINTS], dtype=np.int64)
    seg_b = np.array([j[_SEG_END.get(i, i)] for i in range(NB)])
    return Skeleton(joints=j, parents=parents, seg_a=j.copy(), seg_b=seg_b)


def _axis_angle_matrix(axis: np.ndarray, angle: float) -> np.ndarray:
    a = axis / np.linalg.norm(axis)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * k + (1.0 - math.cos(angle)) * (k @ k)


@dataclasses.dataclass(frozen=True)
class Pose:
    B: np.ndarray      # [NB, 3, 4] rigid bone transforms (canonical -> posed)
    params: np.ndarray  # [NB, 6] axis-angle (3) + translation (3) per bone


def make_pose(skel: Skeleton, seed: int, max_deg: float = 30.0, trans_std: float = 0.02) -> Pose:
    """B_i = T(j_i + t_i) R_i T(-j_i): a rotation about the bone's own rest
    joint, axis uniform on the sphere, angle U(-max_deg, max_deg), translation
    t_i ~ N(0, trans_std^2 I); bones are independent (no forward kinematics)."""
    rng = np.random.default_rng(seed)
    B = np.zeros((NB, 3, 4))
    params = np.zeros((NB, 6))
    for i in range(NB):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        ang = math.radians(rng.uniform(-max_deg, max_deg))
        t = rng.normal(0.0, trans_std, size=3)
        R = _axis_angle_matrix(axis, ang)
        jnt = skel.joints[i]
        B[i, :, :3] = R
        B[i, :, 3] = jnt + t - R @ jnt
        params[i, :3] = axis * ang
        params[i, 3:] = t
    return Pose(B=B, params=params)


def identity_pose(nb: int = NB) -> np.ndarray:
    B = np.zeros((nb, 3, 4))
    B[:, :, :3] = np.eye(3)
    return B


def _seg_dist(p: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    ab = b - a
    den = float(ab @ ab)
    if den == 0.0:
        return np.linalg.norm(p - a, axis=-1)
    t = np.clip(((p - a) @ ab) / den, 0.0, 1.0)
    return np.linalg.norm(p - (a + t[..., None] * ab), axis=-1)


def make_skin_grid(skel: Skeleton, dims: tuple[int, int, int], lo, hi, temp: float = 10.0) -> np.ndarray:
    """Skinning weights at the grid vertices: softmax over bones of
    -temp * (distance from the vertex to the bone's rest segment).
    dims = (Dx, Dy, Dz); vertices sit on the box corners (align-corners).
    Returns [Dz, Dy, Dx, NB] float64."""
    dx, dy, dz = dims
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    xs = lo[0] + (hi[0] - lo[0]) * np.arange(dx) / (dx - 1)
    ys = lo[1] + (hi[1] - lo[1]) * np.arange(dy) / (dy - 1)
    zs = lo[2] + (hi[2] - lo[2]) * np.arange(dz) / (dz - 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    d = np.stack([_seg_dist(P, skel.seg_a[i], skel.seg_b[i]) for i in range(NB)], axis=-1)
    logits = -temp * d
    logits -= logits.max(axis=-1, keepdims=True)
    e = np.exp(logits)
    return e / e.sum(axis=-1, keepdims=True)


def _posed_segments(skel: Skeleton, B: np.ndarray):
    a = np.einsum("nij,nj->ni", B[:, :, :3], skel.seg_a) + B[:, :, 3]
    b = np.einsum("nij,nj->ni", B[:, :, :3], skel.seg_b) + B[:, :, 3]
    return a, b


def _ellipsoid_union(G: int, a: np.ndarray, b: np.ndarray, rho: np.ndarray, s: float) -> np.ndarray:
    occ = np.zeros((G, G, G), dtype=bool)
    h = 1.0 / G
    for i in range(a.shape[0]):
        c = 0.5 * (a[i] + b[i])
        seg = b[i] - a[i]
        L = float(np.linalg.norm(seg))
        u = seg / L if L > 0 else np.array([1.0, 0.0, 0.0])
        r = s * rho[i]
        ax = 0.5 * L + r
        lo = np.clip(np.floor((c - ax) / h).astype(int) - 1, 0, G - 1)
        hi = np.clip(np.ceil((c + ax) / h).astype(int) + 1, 0, G - 1)
        zs = (np.arange(lo[2], hi[2] + 1) + 0.5) * h
        ys = (np.arange(lo[1], hi[1] + 1) + 0.5) * h
        xs = (np.arange(lo[0], hi[0] + 1) + 0.5) * h
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        v = np.stack([X - c[0], Y - c[1], Z - c[2]], axis=-1)
        proj = v @ u
        perp2 = np.maximum((v * v).sum(-1) - proj * proj, 0.0)
        inside = (proj / ax) ** 2 + perp2 / (r * r) <= 1.0
        occ[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] |= inside
    return occ


def make_occupancy(skel: Skeleton, B: np.ndarray, G: int, target: float, seed: int) -> np.ndarray:
    """Union of one ellipsoid per bone around its posed segment (long
    semi-axis |seg|/2 + r_i, the others r_i, r_i = s * rho_i with
    rho_i ~ U(0.6, 1.4)); s is bisected until the occupied fraction of the
    G^3 cell centres is target +- 0.5 %.  Returns bool [G, G, G] indexed
    [z, y, x]."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.6, 1.4, size=NB)
    a, b = _posed_segments(skel, B)
    lo_s, hi_s = 1e-3, 1.0
    occ = None
    for _ in range(60):
        s = 0.5 * (lo_s + hi_s)
        occ = _ellipsoid_union(G, a, b, rho, s)
        frac = occ.mean()
        if abs(frac - target) <= 0.005:
            return occ
        if frac < target:
            lo_s = s
        else:
            hi_s = s
    return occ


def front_face_rays(n: int = 32, cam_z: float = -1.0):
    """n x n pinhole rays from (0.5, 0.5, cam_z) through the pixel centres of
    the unit box's front face z = 0 (every ray enters the box)."""
    o = np.array([0.5, 0.5, cam_z])
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    p = np.stack([(ii + 0.5) / n, (jj + 0.5) / n, np.zeros_like(ii, dtype=np.float64)], -1).reshape(-1, 3)
    d = p - o
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.broadcast_to(o, d.shape).copy(), d


def camera_rays(H: int = 540, W: int = 540, f: float = 583.2, cx: float = 270.0, cy: float = 270.0,
                origin=(0.5, 0.5, -1.2)):
    """Pinhole camera looking along +z; one ray per pixel centre, row-major."""
    o = np.asarray(origin, dtype=np.float64)
    v, u = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    d = np.stack([(u + 0.5 - cx) / f, (v + 0.5 - cy) / f, np.ones((H, W))], -1).reshape(-1, 3)
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.broadcast_to(o, d.shape).copy(), d


def make_hash_table(L: int, T: int, F: int, seed: int = 2, scale: float = 1e-4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(L, T, F))


def make_mlp(widths=(32, 64, 64, 4), seed: int = 3, sigma_bias: float = 0.0, bias_std: float = 0.1) -> np.ndarray:
    """Seeded Gaussian init: He-normal weights N(0, 2/fan_in) and biases
    N(0, bias_std^2) (the density output bias is then set to sigma_bias).
    Non-zero biases keep the hidden pre-activations away from the ReLU kink
    when the hash features are tiny.  Flat layout: for each layer W [out][in]
    row-major, then b [out]."""
    rng = np.random.default_rng(seed)
    parts = []
    for li in range(len(widths) - 1):
        fi, fo = widths[li], widths[li + 1]
        Wl = rng.normal(0.0, math.sqrt(2.0 / fi), size=(fo, fi))
        bl = rng.normal(0.0, bias_std, size=fo)
        if li == len(widths) - 2:
            bl[0] = sigma_bias
        parts += [Wl.ravel(), bl]
    return np.concatenate(parts)


def hash_resolution_params():
    """Base resolution and per-level growth factor of the multiresolution grid."""
    return 16.0, 1.38


@dataclasses.dataclass
class Workload:
    """One seeded configuration, every array already in its storage dtype."""
    name: str
    rays_o: np.ndarray      # [R, 3] f32
    rays_d: np.ndarray      # [R, 3] f32
    occ: np.ndarray | None  # [G, G, G] u8 (z, y, x) or None (no skipping)
    occ_aabb: np.ndarray    # [6] f32 (lo xyz, hi xyz)
    dt: float               # uniform step (0 -> use n_per_ray)
    n_per_ray: int          # fixed samples per chord (0 -> use dt)
    max_steps: int
    B: np.ndarray           # [NB, 3, 4] f32
    pose_params: np.ndarray  # [NB, 6] f32
    W: np.ndarray           # [Dz, Dy, Dx, NB] f32
    skin_aabb: np.ndarray   # [6] f32
    hash_aabb: np.ndarray   # [6] f32
    table: np.ndarray       # [L, T, F] f32 master
    L: int
    F: int
    log2T: int
    mlp: np.ndarray         # flat f32
    widths: tuple
    max_iter: int
    tol_stop: float
    tol_valid: float
    T_thresh: float
    target: np.ndarray | None  # [R, 3] f32
    base_res: float = 16.0
    growth: float = 1.38

    @property
    def R(self) -> int:
        return self.rays_o.shape[0]


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


@functools.lru_cache(maxsize=None)
def _skeleton_cached(seed):
    return make_skeleton(seed)


@functools.lru_cache(maxsize=8)
def _skin_cached(dims, lo, hi):
    return make_skin_grid(_skeleton_cached(0), dims, lo, hi)


@functools.lru_cache(maxsize=16)
def _occ_cached(pose_seed, G, target, seed):
    skel = _skeleton_cached(0)
    pose = make_pose(skel, pose_seed)
    return make_occupancy(skel, pose.B, G, target, seed)


def tiny_forward(pose_seed: int = 1) -> Workload:
    """Plain FP32 forward, tiny: 32^3 x 24 skinning grid over the unit box,
    1024 front-face rays x 64 uniform samples, no occupancy grid, hash
    T = 2^14, MLP 32-64-64-4, Broyden <= 10 iterations, 24 inits."""
    skel = _skeleton_cached(0)
    pose = make_pose(skel, pose_seed)
    o, d = front_face_rays(32)
    box = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    return Workload(
        name="tiny_fwd_f32", rays_o=_f32(o), rays_d=_f32(d), occ=None, occ_aabb=_f32(box),
        dt=0.0, n_per_ray=64, max_steps=64, B=_f32(pose.B), pose_params=_f32(pose.params),
        W=_f32(_skin_cached((32, 32, 32), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))), skin_aabb=_f32(box),
        hash_aabb=_f32(box), table=_f32(make_hash_table(16, 1 << 14, 2)), L=16, F=2, log2T=14,
        mlp=_f32(make_mlp()), widths=(32, 64, 64, 4), max_iter=10, tol_stop=1e-6, tol_valid=1e-5,
        T_thresh=0.0, target=None)


def _body_frame(name, n_rays, occ_frac, pose_seed, ray_seed, target_seed, sigma_bias, T_thresh,
                table_scale, res=540):
    skel = _skeleton_cached(0)
    pose = make_pose(skel, pose_seed)
    # the 540^2 camera's field of view at any resolution
    o, d = camera_rays(res, res, 583.2 * (res / 540.0), res / 2.0, res / 2.0)
    if n_rays < o.shape[0]:
        idx = np.sort(np.random.default_rng(ray_seed).choice(o.shape[0], size=n_rays, replace=False))
        o, d = o[idx], d[idx]
    target = None
    if target_seed is not None:
        target = _f32(np.random.default_rng(target_seed).uniform(0.0, 1.0, size=(n_rays, 3)))
    box = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    return Workload(
        name=name, rays_o=_f32(o), rays_d=_f32(d),
        occ=_occ_cached(pose_seed, 128, occ_frac, 7).astype(np.uint8), occ_aabb=_f32(box),
        dt=float(np.float32(math.sqrt(3.0) / 128.0)), n_per_ray=0, max_steps=128,
        B=_f32(pose.B), pose_params=_f32(pose.params),
        W=_f32(_skin_cached((64, 64, 32), (0.0, 0.0, 0.25), (1.0, 1.0, 0.75))),
        skin_aabb=_f32((0.0, 0.0, 0.25, 1.0, 1.0, 0.75)), hash_aabb=_f32(box),
        table=_f32(make_hash_table(16, 1 << 19, 2, scale=table_scale)), L=16, F=2, log2T=19,
        mlp=_f32(make_mlp(sigma_bias=sigma_bias)), widths=(32, 64, 64, 4), max_iter=10,
        tol_stop=1e-6, tol_valid=1e-5, T_thresh=T_thresh, target=target)


def train_step(pose_seed: int = 1, table_scale: float = 1e-4) -> Workload:
    """Training step: 8192 random pixels of the 540^2 camera, <= 128 samples
    per ray through a 128^3 occupancy grid (~15 % occupied), 64x64x32x24
    skinning grid, hash T = 2^19, L2 loss against U[0,1]^3 targets."""
    return _body_frame("train_step", 8192, 0.15, pose_seed, 4, 5, 0.0, 0.0, table_scale)


def full_frame(pose_seed: int = 1, table_scale: float = 1e-4) -> Workload:
    """Full-frame inference: 540 x 540 rays, ~10 % occupancy, early ray
    termination at transmittance 1e-4, density output bias +4."""
    return _body_frame("frame540", 540 * 540, 0.10, pose_seed, None, None, 4.0, 1e-4, table_scale)


def folded_pose(skel: Skeleton, bone: int = 4, deg: float = 120.0) -> np.ndarray:
    """Rest pose except one bone turned by `deg` about the z axis through its
    rest joint (a fold in the body's plane): with sharp skinning weights,
    posed points near the fold have a root in each of the two overlapping
    parts (several canonical correspondences, Sec. 3.1)."""
    B = identity_pose()
    a = math.radians(deg)
    R = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
    j = skel.joints[bone]
    B[bone, :, :3] = R
    B[bone, :, 3] = j - R @ j
    return B


@functools.lru_cache(maxsize=2)
def _folded_cached(res, temp):
    skel = _skeleton_cached(0)
    B = folded_pose(skel)
    W = make_skin_grid(skel, (64, 64, 32), (0.0, 0.0, 0.25), (1.0, 1.0, 0.75), temp=temp)
    occ = make_occupancy(skel, B, 128, 0.10, 7)
    return B, W, occ


def folded_frame(res: int = 540, table_scale: float = 1e-4, temp: float = 100.0) -> Workload:
    """A frame of a folded pose (one leg bone turned 120 degrees in the body's
    plane) with sharp skinning weights (softmax temperature 100): about 6 % of
    the posed points near the body have two distinct roots.  The 540^2
    camera's field of view, ~10 % occupancy built from the folded pose, no
    termination, density output bias 0."""
    B, W, occ = _folded_cached(res, temp)
    o, d = camera_rays(res, res, 583.2 * (res / 540.0), res / 2.0, res / 2.0)
    box = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    return Workload(
        name=f"folded{res}", rays_o=_f32(o), rays_d=_f32(d), occ=occ.astype(np.uint8), occ_aabb=_f32(box),
        dt=float(np.float32(math.sqrt(3.0) / 128.0)), n_per_ray=0, max_steps=128,
        B=_f32(B), pose_params=np.zeros((NB * 6,), np.float32),
        W=_f32(W), skin_aabb=_f32((0.0, 0.0, 0.25, 1.0, 1.0, 0.75)), hash_aabb=_f32(box),
        table=_f32(make_hash_table(16, 1 << 19, 2, scale=table_scale)), L=16, F=2, log2T=19,
        mlp=_f32(make_mlp()), widths=(32, 64, 64, 4), max_iter=10,
        tol_stop=1e-6, tol_valid=1e-5, T_thresh=0.0, target=None)


BATCH_RES = (270, 540, 1080)


def batch_pose(k: int, n: int = 16, table_scale: float = 1e-4) -> Workload:
    """Pose k of the batched render: pose seed 3000 + k, occupancy
    5 % + 20 % k / (n - 1), resolution 270^2, 540^2 or 1080^2 by k mod 3
    (the 540^2 camera's field of view), termination at T < 1e-4, density
    output bias +4.  One avatar: the hash table, MLP and skinning grid are
    those of full_frame."""
    frac = 0.05 + 0.20 * k / max(n - 1, 1)
    res = BATCH_RES[k % 3]
    return _body_frame(f"batch{k}", res * res, frac, 3000 + k, None, None, 4.0, 1e-4, table_scale, res=res)


def batch_poses(n: int = 16, table_scale: float = 1e-4, workers: int = 1) -> list:
    """The n poses of the batched render (occupancy grids built in a process
    pool of `workers` when > 1)."""
    if workers > 1:
        import concurrent.futures as cf
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(batch_pose, range(n), [n] * n, [table_scale] * n))
    return [batch_pose(k, n, table_scale) for k in range(n)]


def ray_subset(w: Workload, idx: np.ndarray) -> Workload:
    """The same workload restricted to the rays ``idx`` (for oracle-sized checks)."""
    idx = np.asarray(idx)
    return dataclasses.replace(
        w, rays_o=np.ascontiguousarray(w.rays_o[idx]), rays_d=np.ascontiguousarray(w.rays_d[idx]),
        target=None if w.target is None else np.ascontiguousarray(w.target[idx]))


def random_points(n: int, seed: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Uniform points in a box, [n, 3] float32."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo)
    hi = np.asarray(hi)
    return _f32(lo + (hi - lo) * rng.uniform(size=(n, 3)))


def make_rootinit_params(nb: int = NB, hidden: int = 64, seed: int = 11) -> np.ndarray:
    """He-normal initial weights of the root-initialiser MLP
    (3 + 6 nb) -> hidden -> hidden -> (nb + 3), zero biases; flat layout as
    make_mlp."""
    return make_mlp((3 + 6 * nb, hidden, hidden, nb + 3), seed=seed, bias_std=0.0)


def sample_posed_points(skel: Skeleton, B: np.ndarray, n: int, seed: int, radius: float = 0.05) -> np.ndarray:
    """n points uniform in the union of capsules of the given radius around
    the posed bone segments (rejection sampling in their bounding box)."""
    rng = np.random.default_rng(seed)
    a, b = _posed_segments(skel, B)
    lo = np.minimum(a, b).min(0) - radius
    hi = np.maximum(a, b).max(0) + radius
    out = []
    got = 0
    while got < n:
        p = lo + (hi - lo) * rng.uniform(size=(4 * n, 3))
        d = np.min(np.stack([_seg_dist(p, a[i], b[i]) for i in range(a.shape[0])], -1), -1)
        p = p[d <= radius]
        out.append(p)
        got += p.shape[0]
    return _f32(np.concatenate(out)[:n])
