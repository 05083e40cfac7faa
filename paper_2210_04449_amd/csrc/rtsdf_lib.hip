// The library's main translation unit: every .hip file of this directory but
// jfa.hip, so device globals (the error word, the empty brick) need no
// relocatable device code.  jfa.hip is a unit of its own (its device code is
// built without NaN semantics); nothing here calls its kernels, and the
// batched JFA kernel takes the pass bodies from jfa_device.hpp.
#include "api.hip"
#include "voxelize.hip"
#include "select.hip"
#include "scene.hip"
#include "instance.hip"
#include "trace.hip"
#include "lbvh.hip"
#include "distance.hip"
#include "shadow.hip"
#include "batch.hip"
#include "graph.hip"
